// Bottom level of the pyramid (Sec. 3.2, Eqs. (3)-(4), Algorithm 1):
//   A_0(p, q) = 1/16 sum_{4x4 offsets d} <D1[p+d], D2[q+d]>   (D2 = 0 outside I')
//   C_0 = max(A_0, 0)^lambda,  C'_0 = (S o P)(C_0) with argmax codes (Eqs. (8)-(9)).
//
// The correlation is an implicit GEMM on the matrix cores: M = atomic
// patches, N = target positions, K = 16 offsets x 9 channels.  The K order is
// chosen so that each 16-lane group of a wave owns one row of the 4x4 patch:
// its K slice is 4 consecutive pixels x channels, i.e. one contiguous run in
// the HWC descriptor layout for both operands.  Patch fragments stay in
// registers for the whole block; the target tile sits in LDS.
//
// Epilogue: the 3x3/stride-2 max-pool with its first-maximum argmax and the
// rectification are fused, so C_0 itself is never written.  Because x^lambda
// is increasing on [0, inf), the pool runs on max(A, 0) and only the pooled
// value is raised to lambda.
//
// Block = 4 waves; each wave owns 2 M-tiles of 16 patches (128 patches per
// block).  A block owns a band of TR pooled rows and sweeps it from left to
// right, 16 pooled columns per step.  Per A-row it computes two N-tiles: the
// even positions x = 2c and the odd positions x = 2c+1 of the 16 columns c,
// so pooled column c needs O[c-1], E[c], O[c]: O[c-1] comes from the
// neighbouring lane (DPP row shift) or, for the first column of a step, from
// the previous step (a per-row carry in LDS).  Every pooled row of a patch is
// then written as one aligned 16-float run, and consecutive steps complete
// the same cache lines.
#include "dm_group.h"

namespace dm {
namespace {

constexpr int MT = 2;                // BF16: M-tiles (16 patches) per wave
constexpr int MF = 1;                // FP32: M-tiles per wave (its register budget allows three waves per SIMD)
constexpr int WAVES = 4;
constexpr int PT = 16 * MT * WAVES;  // BF16: patches per block
constexpr int PF = 16 * MF * WAVES;  // FP32: patches per block
constexpr int TR = 8;                // pooled rows per band
constexpr int ARS = 2 * TR + 1;      // A-rows per band
constexpr int D2R = 2 * TR + 4;      // target tile rows (A-rows + patch height - 1)
constexpr int D2C = 35;              // target tile columns: 2C0-2 .. 2C0+32

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct PoolArgs {
    int natom, n0x, W1, W2, H2, h1, w1;
    int pos;                // correlations inside I' are positive and normal (Geom::pos_corr)
    int n_ptiles, n_steps;
    int n_seg, seg_steps;   // column segments of n_steps / n_seg steps (few patches: more blocks)
};

// Steps [s_begin, s_end) a block computes and the first one it stores: a
// segment after the first starts one step early, so that the carry (the odd
// column left of its first pooled column) is computed rather than unknown.
struct StepRange {
    int s_begin, s_out, s_end;
};
__device__ inline StepRange step_range(const PoolArgs& a, int seg) {
    const int s0 = seg * a.seg_steps;
    return StepRange{s0 > 0 ? s0 - 1 : 0, s0, min(a.n_steps, s0 + a.seg_steps)};
}

// Lane n of each 16-lane row receives v from lane n-1; lane 0 receives `first`.
__device__ inline float shift_in(float v, float first) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(v), 0x111, 0xF, 0xF,
                                                      false));
}

__device__ inline bf8 load_bf8(const uint32_t* p) {
    union {
        uint32_t u[4];
        bf8 v;
    } x;
    x.u[0] = p[0];
    x.u[1] = p[1];
    x.u[2] = p[2];
    x.u[3] = p[3];
    return x.v;
}

// Two packed bf16 values times 1/16: an exponent shift, exact for normal
// values (zero stays zero; values below 2^-122 would flush to zero).
__device__ inline uint32_t bf16x2_scale16(uint32_t u) {
    uint32_t r = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t b = (u >> (16 * h)) & 0xFFFFu;
        const uint32_t e = (b >> 7) & 0xFFu;
        const uint32_t v = e > 4 ? b - (4u << 7) : (b & 0x8000u);
        r |= v << (16 * h);
    }
    return r;
}

// One x-step of the FP32 sweep.  Engine supplies the MFMA chain for an N-tile
// (E or O) of all MF M-tiles.  POS: correlations inside I' are known
// positive (PoolArgs::pos), so the clamp at 0 is left out.
template <bool POS, typename Engine>
__device__ inline void sweep_band(const Engine& eng, const PoolArgs& a, int pt, int R0, int seg, float lam,
                                  float* __restrict__ cp, uint8_t* __restrict__ code,
                                  float (*carry)[16 * MF]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, grp = lane >> 4;
    const int pbase = pt * PF + wave * 16 * MF;
    // Output offsets of this lane's 4*MF patches (a patch map is h1 x w1).
    size_t obase[MF][4];
#pragma unroll
    for (int mt = 0; mt < MF; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) obase[mt][j] = (size_t)(pbase + mt * 16 + 4 * grp + j) * a.h1 * a.w1;
    const StepRange sr = step_range(a, seg);
    for (int step = sr.s_begin; step < sr.s_end; ++step) {
        const int C0 = 16 * step;
        const bool store = step >= sr.s_out;
        __syncthreads();                         // previous tile fully consumed
        eng.load_tile(a, R0, C0);
        __syncthreads();
        const int c = C0 + n;
        const bool e_ok = 2 * c < a.W2, o_ok = 2 * c + 1 < a.W2;
        float best[MF][4];
        int bk[MF][4];
        for (int ia = 0; ia < ARS; ++ia) {
            const int y = 2 * R0 - 1 + ia;
            const bool y_ok = y >= 0 && y < a.H2;
            f4 accE[MF], accO[MF];
            eng.mfma_row(ia, 2 * n, accE);
            eng.mfma_row(ia, 2 * n + 1, accO);
#pragma unroll
            for (int mt = 0; mt < MF; ++mt) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int lp = mt * 16 + 4 * grp + j;
                    const float E = (y_ok && e_ok) ? (POS ? accE[mt][j] : fmaxf(accE[mt][j], 0.f)) : -1.f;
                    const float O = (y_ok && o_ok) ? (POS ? accO[mt][j] : fmaxf(accO[mt][j], 0.f)) : -1.f;
                    const float cin = step > sr.s_begin ? carry[ia][lp] : -1.f;   // O of column C0-1
                    const float L = shift_in(O, cin);
                    if (n == 15) carry[ia][lp] = O;
                    // row maximum, first in order mx = -1, 0, +1
                    float rm = L;
                    int rk = 0;
                    if (E > rm) {
                        rm = E;
                        rk = 1;
                    }
                    if (O > rm) {
                        rm = O;
                        rk = 2;
                    }
                    if (ia & 1) {                              // my = 0 of pooled row R0 + ia/2
                        if (rm > best[mt][j]) {
                            best[mt][j] = rm;
                            bk[mt][j] = 3 + rk;
                        }
                    } else {
                        if (ia > 0) {                          // my = +1: finish pooled row R0 + ia/2 - 1
                            float bv = best[mt][j];
                            int bc = bk[mt][j];
                            if (rm > bv) {
                                bv = rm;
                                bc = 6 + rk;
                            }
                            const int r = R0 + ia / 2 - 1, jp = pbase + lp;
                            if (store && r < a.h1 && c < a.w1 && jp < a.natom) {
                                const size_t o = obase[mt][j] + (uint32_t)(r * a.w1 + c);
                                cp[o] = rect_pow(bv, lam);
                                code[o] = (uint8_t)bc;
                            }
                        }
                        best[mt][j] = rm;                      // my = -1 of pooled row R0 + ia/2
                        bk[mt][j] = rk;
                    }
                }
            }
        }
    }
}

struct EngineF32 {
    const float* fa;   // [MF][36] patch fragments (registers of the caller)
    float* sD2;        // [D2R][D2C][9]
    const float* d2;
    __device__ void load_tile(const PoolArgs& a, int R0, int C0) const {
        const int ybase = 2 * R0 - 3, xbase = 2 * C0 - 2;
        for (int e = threadIdx.x; e < D2R * D2C * 9; e += 256) {
            const int row = e / (D2C * 9), rem = e - row * (D2C * 9);
            const int y = ybase + row, x = xbase + rem / 9, ch = rem % 9;
            sD2[e] = (y >= 0 && y < a.H2 && x >= 0 && x < a.W2) ? d2[((size_t)y * a.W2 + x) * 9 + ch] : 0.f;
        }
    }
    // A on A-row ia for the 16 positions whose tile column (minus 2) is col0 + 2*lane.
    __device__ void mfma_row(int ia, int col, f4* acc) const {
        const int grp = (threadIdx.x & 63) >> 4;
        const float* bs = sD2 + ((ia + grp) * D2C + col) * 9;
        float fb[36];
#pragma unroll
        for (int t = 0; t < 36; ++t) fb[t] = bs[t];
#pragma unroll
        for (int mt = 0; mt < MF; ++mt) {
            f4 r = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 36; ++t) r = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[mt * 36 + t], fb[t], r, 0, 0, 0);
            acc[mt] = r;
        }
    }
};

// The lane's run of target words at A-row ia starts at pixel 2n (even
// column) and, one pixel (5 words) on, at pixel 2n + 1 (odd column).  The even
// MFMAs take run words 0..19 as quads {0-3} ... {16-19} against patch words in
// the same order (fa).  The odd run is words 5..24: three of its quads are the
// even run's {8-11}, {12-15}, {16-19}, reused as they are, and two more are
// loaded, {5, 6, 7, 20} and {21-24}; faO holds the patch words in that order
// (run word w pairs with patch word w - 5).
struct EngineBF16 {
    const bf8* fa;     // [MT][5]
    const bf8* faO;    // [MT][5], K order of the odd run
    uint32_t* sD2;     // [D2R][D2C][5] bf16 pairs
    const uint32_t* d2;
    __device__ void load_tile(const PoolArgs& a, int R0, int C0) const {
        const int ybase = 2 * R0 - 3, xbase = 2 * C0 - 2;
        for (int e = threadIdx.x; e < D2R * D2C * 5; e += 256) {
            const int row = e / (D2C * 5), rem = e - row * (D2C * 5);
            const int y = ybase + row, x = xbase + rem / 5, pr = rem % 5;
            sD2[e] = (y >= 0 && y < a.H2 && x >= 0 && x < a.W2) ? d2[((size_t)y * a.W2 + x) * 5 + pr] : 0u;
        }
    }
    // Even (accE) and odd (accO) columns of A-row ia for the lane's patches.
    __device__ void mfma_row(int ia, f4* accE, f4* accO) const {
        const int grp = (threadIdx.x & 63) >> 4, n = threadIdx.x & 15;
        const uint32_t* bs = sD2 + ((ia + grp) * D2C + 2 * n) * 5;
        bf8 fb[7];
#pragma unroll
        for (int s = 0; s < 5; ++s) fb[s] = load_bf8(bs + 4 * s);
        {
            union {
                uint32_t u[4];
                bf8 v;
            } x;
            x.u[0] = bs[5];
            x.u[1] = bs[6];
            x.u[2] = bs[7];
            x.u[3] = bs[20];
            fb[5] = x.v;
        }
        fb[6] = load_bf8(bs + 21);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f4 r = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 5; ++s) r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[mt * 5 + s], fb[s], r, 0, 0, 0);
            accE[mt] = r;
            f4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 5; ++s)
                q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(faO[mt * 5 + s], fb[s + 2], q, 0, 0, 0);
            accO[mt] = q;
        }
    }
};

// ---------------------------------------------------------------- BF16 sweep
// Same band and step order as sweep_band, with two changes.
//
// Target tile: a tile row is one contiguous run of D2C pixels x 5 words of
// the HWC bf16 layout, so each thread owns fixed (row, word) slots; the next
// step's tile is fetched into registers while the current one is computed.
//
// Packed-key epilogue: each rectified value v (clamped below at 2^-126, whose
// power is 0 in FP32 like that of 0) becomes the key
//   (bits(v) with the low 4 mantissa bits cleared) | (15 - k)
// for window position k.  Non-negative floats order like their bit patterns,
// so the max over keys is the max over values, with equal values (and values
// within 2^-19 of each other) going to the first position k: every pool
// comparison is one integer max.  Positions outside I' keep only the position
// bits and lose against every valid key.  The pooled value is the kept
// 19-bit-mantissa maximum, well inside the rounding of the BF16 operands.
constexpr int TILE_W = D2C * 5;                          // words per tile row
constexpr int TILE_N = D2R * TILE_W;                     // words per tile
constexpr int TILE_PER_T = (TILE_N + 255) / 256;         // words per thread
constexpr int kOOB = 0x7ffffff0;                         // buffer byte offset past any buffer
// Codes of two steps (32 pooled columns) of a wave's 16 MT patches x TR rows,
// staged in LDS and written as 16-byte runs (a 32-byte sector per patch row)
// when the pooled width is a multiple of 16: one step's 16 codes alone
// leave half-written sectors, which HBM writes whole.
constexpr int kKRow = 32;                                // bytes per staged row (two steps)
constexpr int kKStride = TR * kKRow + 16;                // bytes per patch (padded: other banks)

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}

// Keys of A-row ia of the step for this lane's 4 * MT patches: the row
// maximum over the window columns k = 0, 1, 2 (odd column left of the lane's
// pooled column, even column, odd column), each carrying bits - k, where
// bits = 15 - 3 (my + 1) places the row in the window.  The carry (keys of
// the odd column left of the step) moves through LDS 4 values at a time.
// POS: correlations inside I' are known positive and normal, so the clamp
// at 2^-126 changes nothing and is left out.
template <bool POS>
__device__ __forceinline__ void row_keys(const EngineBF16& eng, const PoolArgs& a, int R0, int ia, int n,
                                         uint32_t me, uint32_t mo, uint32_t bits, const float* cr, float* cw,
                                         uint32_t (&rk)[MT][4]) {
    const int y = 2 * R0 - 1 + ia;
    const bool y_ok = y >= 0 && y < a.H2;
    const uint32_t mE = y_ok ? me : 0u, mO = y_ok ? mo : 0u;
    const int lo = 0x00800000;   // bits of 2^-126; as signed integers, floats below it (negatives too) are smaller
    f4 accE[MT], accO[MT];
    eng.mfma_row(ia, accE, accO);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const f4 cin = *reinterpret_cast<const f4*>(__builtin_assume_aligned(cr + mt * 16, 16));   // O of column C0-1
        f4 kout;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int bE = __float_as_int(accE[mt][j]), bO = __float_as_int(accO[mt][j]);
            const uint32_t kE = ((uint32_t)(POS ? bE : max(bE, lo)) & mE) | (bits - 1u);   // k = 1
            const uint32_t kO = ((uint32_t)(POS ? bO : max(bO, lo)) & mO) | (bits - 2u);   // k = 2
            const uint32_t kL =
                ((uint32_t)__builtin_amdgcn_update_dpp((int)__float_as_uint(cin[j]), (int)kO, 0x111, 0xF, 0xF, false) &
                 ~15u) | bits;                                                                          // k = 0
            kout[j] = __uint_as_float(kO);
            rk[mt][j] = max(max(kL, kE), kO);
        }
        *reinterpret_cast<f4*>(__builtin_assume_aligned(cw + mt * 16, 16)) = kout;
    }
}

// STAGE: the pooled width is a multiple of 16, codes go out through sK.
// POS: see row_keys.
template <bool STAGE, bool POS>
__device__ inline void sweep_band_bf16(const bf8* fa, const bf8* faO, uint32_t* sD2, const uint32_t* __restrict__ d2,
                                       const PoolArgs& a, int pt, int R0, int seg, float lam, float* __restrict__ cp,
                                       uint8_t* __restrict__ code, float (*carry)[16 * MT], float* dummy,
                                       uint8_t* __restrict__ sK) {
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = lane & 15, grp = lane >> 4;
    const int pbase = pt * PT + wave * 16 * MT;
    const uint32_t mapsz = (uint32_t)a.h1 * a.w1;
    // Output buffers of this wave's patches: patches past natom are out of range.
    const uint32_t nmap = __builtin_amdgcn_readfirstlane(max(0, min(16 * MT, a.natom - pbase)) * (int)mapsz);
    const auto rsC = buf_rsrc(cp + (size_t)pbase * mapsz, nmap * 4);
    const auto rsK = buf_rsrc(code + (size_t)pbase * mapsz, nmap);
    const auto rsD = buf_rsrc(d2, (uint32_t)a.H2 * a.W2 * 20);
    // Tile slots of this thread: words tid + 256 it of the tile (row-major,
    // TILE_W words per row), recomputed at each fetch to keep registers free.
    const int ybase = 2 * R0 - 3;
    uint32_t tv[TILE_PER_T];
    auto fetch = [&](int C0) {
        const int xw = (2 * C0 - 2) * 5;   // word offset of the tile's first pixel within a row
#pragma unroll
        for (int it = 0; it < TILE_PER_T; ++it) {
            const int idx = tid + 256 * it, row = idx / TILE_W, w = xw + idx - row * TILE_W, y = ybase + row;
            const bool ok = idx < TILE_N && y >= 0 && y < a.H2 && w >= 0 && w < a.W2 * 5;
            tv[it] = __builtin_amdgcn_raw_buffer_load_b32(rsD, ok ? (y * a.W2 * 5 + w) * 4 : kOOB, 0, 0);
        }
    };
    // Carry (key of the odd column left of the step) starts as "outside".
#pragma unroll
    for (int e = lane; e < ARS * 16 * MT; e += 64) (&carry[0][0])[e] = 0.f;
    // Lanes other than n = 15 write their carry into a private dummy slot
    // (16-byte aligned, 4 words per lane and M-tile).
    float* const cw0 = n == 15 ? &carry[0][4 * grp] : dummy + 4 * lane;
    const int cstep = n == 15 ? 16 * MT : 0;
    // Output offsets (pooled row 0, column n) of this lane's 4 * MT patches,
    // in bytes for the codes and for the values; the row and step part of an
    // offset is uniform and goes into the instruction's scalar offset.
    // Patches past natom get offsets past the end of the buffers, so their
    // stores are dropped.
    uint32_t ob[MT][4], ob4[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t lp = mt * 16 + 4 * grp + j;
            const bool ok = lp * mapsz < nmap;
            ob[mt][j] = ok ? lp * mapsz + n : (uint32_t)kOOB;
            ob4[mt][j] = ok ? (lp * mapsz + n) * 4 : (uint32_t)kOOB;
        }
    const StepRange sr = step_range(a, seg);
    fetch(16 * sr.s_begin);
    for (int step = sr.s_begin; step < sr.s_end; ++step) {
        const int C0 = 16 * step;
        __syncthreads();                         // previous tile fully consumed
#pragma unroll
        for (int it = 0; it < TILE_PER_T; ++it) {
            const int idx = tid + 256 * it;
            if (idx < TILE_N) sD2[idx] = tv[it];
        }
        __syncthreads();
        if (step + 1 < sr.s_end) fetch(C0 + 16);
        const EngineBF16 eng{fa, faO, sD2, d2};
        const int c = C0 + n;
        const uint32_t me = 2 * c < a.W2 ? ~15u : 0u, mo = 2 * c + 1 < a.W2 ? ~15u : 0u;
        uint32_t best[MT][4], rk[MT][4];
        row_keys<POS>(eng, a, R0, 0, n, me, mo, 15u, carry[0] + 4 * grp, cw0, rk);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) best[mt][j] = rk[mt][j];   // my = -1 of pooled row R0
        for (int pr = 0; pr < TR; ++pr) {
            const int r = R0 + pr;
            row_keys<POS>(eng, a, R0, 2 * pr + 1, n, me, mo, 12u, carry[2 * pr + 1] + 4 * grp, cw0 + (2 * pr + 1) * cstep,
                     rk);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) best[mt][j] = max(best[mt][j], rk[mt][j]);   // my = 0
            row_keys<POS>(eng, a, R0, 2 * pr + 2, n, me, mo, 9u, carry[2 * pr + 2] + 4 * grp, cw0 + (2 * pr + 2) * cstep,
                     rk);
            uint32_t fin[MT][4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    fin[mt][j] = max(best[mt][j], rk[mt][j]);   // my = +1 finishes pooled row r
                    best[mt][j] = rk[mt][j] + 6u;               // the same keys as my = -1 of pooled row r + 1
                }
            if (step >= sr.s_out && r < a.h1 && c < a.w1) {
                const int rc = __builtin_amdgcn_readfirstlane(r * a.w1 + C0);   // uniform part of the offsets
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        __builtin_amdgcn_raw_buffer_store_b32(
                            // the kept value is >= 2^-126 > 0: the power needs no test for 0
                            __float_as_uint(__builtin_amdgcn_exp2f(lam * __builtin_amdgcn_logf(
                                __uint_as_float(fin[mt][j] & ~15u)))), rsC,
                            (int)ob4[mt][j], 4 * rc, 0);
                        const uint8_t k = (uint8_t)(15u - (fin[mt][j] & 15u));
                        if constexpr (STAGE)
                            sK[(mt * 16 + 4 * grp + j) * kKStride + pr * kKRow + (step & 1) * 16 + n] = k;
                        else
                            __builtin_amdgcn_raw_buffer_store_b8(k, rsK, (int)ob[mt][j], rc, 0);
                    }
            }
        }
        // After the second step of a pair (or the last step): the staged
        // codes go out, lane pairs writing a patch row's 32 bytes.  Only this
        // wave wrote its area, and a wave's LDS accesses complete in order.
        if (STAGE && ((step & 1) || step + 1 == sr.s_end)) {
            const int s0 = step & ~1;
#pragma unroll
            for (int i = 0; i < 16 * MT * TR * 2 / 64; ++i) {
                const int e = lane + 64 * i, lp = e >> 4, pr = (e >> 1) & (TR - 1), hf = e & 1;
                const int st = s0 + hf, r = R0 + pr, col = 16 * st;
                const auto v = *reinterpret_cast<const __attribute__((ext_vector_type(4))) uint32_t*>(
                    __builtin_assume_aligned(sK + lp * kKStride + pr * kKRow + hf * 16, 16));
                // patches past natom lie past the descriptor's range: dropped
                if (st >= sr.s_out && st <= step && r < a.h1 && col < a.w1)
                    __builtin_amdgcn_raw_buffer_store_b128(v, rsK, (int)((uint32_t)lp * mapsz + r * a.w1 + col), 0, 0);
            }
        }
    }
}

__device__ inline void corr_f32_body(const float* __restrict__ d1, const float* __restrict__ d2, const PoolArgs& a,
                                     float lam, float* __restrict__ cp, uint8_t* __restrict__ code, int bid) {
    __shared__ float sD2[D2R * D2C * 9];
    __shared__ float sCarry[WAVES][ARS][16 * MF];
    const int pt = bid % a.n_ptiles, rest = bid / a.n_ptiles;
    const int seg = rest % a.n_seg, R0 = (rest / a.n_seg) * TR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, grp = lane >> 4;
    // Patch fragments: lane (n, grp) holds row grp of the 4x4 patch of patch
    // pbase + 16 mt + n: 4 pixels x 9 channels, contiguous in D1.
    float fa[MF * 36];
#pragma unroll
    for (int mt = 0; mt < MF; ++mt) {
        const int j = pt * PF + wave * 16 * MF + mt * 16 + n;
        if (j < a.natom) {
            const int b = j / a.n0x, aa = j - b * a.n0x;
            const float* src = d1 + ((size_t)(4 * b + grp) * a.W1 + 4 * aa) * 9;
#pragma unroll
            for (int t = 0; t < 36; ++t) fa[mt * 36 + t] = src[t] * 0.0625f;   // the 1/16 of Eq. (3), exact
        } else {
#pragma unroll
            for (int t = 0; t < 36; ++t) fa[mt * 36 + t] = 0.f;
        }
    }
    EngineF32 eng{fa, sD2, d2};
    if (a.pos) sweep_band<true>(eng, a, pt, R0, seg, lam, cp, code, sCarry[wave]);
    else sweep_band<false>(eng, a, pt, R0, seg, lam, cp, code, sCarry[wave]);
}

// BF16 variant: descriptors stored as H x W x 10 bf16 (9 channels + a zero),
// so each 16-lane group's K slice is 4 pixels x 10 = 40 values = 5 steps of
// the 16x16x32 MFMA (K = 160, of which 16 are zero pads).
__device__ inline void corr_bf16_body(const uint16_t* __restrict__ d1, const uint16_t* __restrict__ d2,
                                      const PoolArgs& a, float lam, float* __restrict__ cp,
                                      uint8_t* __restrict__ code, int bid) {
    __shared__ __align__(16) uint32_t sD2[D2R * D2C * 5];
    __shared__ __align__(16) float sCarry[WAVES][ARS][16 * MT];
    __shared__ __align__(16) float sDummy[WAVES][4 * 64 + 16 * MT];   // carry writes of lanes other than the row's last
    __shared__ __align__(16) uint8_t sK[WAVES][16 * MT * kKStride];    // staged codes
    const int pt = bid % a.n_ptiles, rest = bid / a.n_ptiles;
    const int seg = rest % a.n_seg, R0 = (rest / a.n_seg) * TR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, grp = lane >> 4;
    bf8 fa[MT * 5], faO[MT * 5];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int j = pt * PT + wave * 16 * MT + mt * 16 + n;
        uint32_t tmp[20];
        if (j < a.natom) {
            const int b = j / a.n0x, aa = j - b * a.n0x;
            const uint32_t* src = (const uint32_t*)(d1 + ((size_t)(4 * b + grp) * a.W1 + 4 * aa) * 10);
#pragma unroll
            for (int t = 0; t < 20; ++t) tmp[t] = src[t];
        } else {
#pragma unroll
            for (int t = 0; t < 20; ++t) tmp[t] = 0u;
        }
#pragma unroll
        for (int t = 0; t < 20; ++t) tmp[t] = bf16x2_scale16(tmp[t]);   // the 1/16 of Eq. (3)
#pragma unroll
        for (int s = 0; s < 5; ++s) fa[mt * 5 + s] = load_bf8(tmp + 4 * s);
        // The odd run's K order: patch words {3-6}, {7-10}, {11-14}, {0, 1, 2, 15}, {16-19}.
        faO[mt * 5 + 0] = load_bf8(tmp + 3);
        faO[mt * 5 + 1] = load_bf8(tmp + 7);
        faO[mt * 5 + 2] = load_bf8(tmp + 11);
        {
            const uint32_t q[4] = {tmp[0], tmp[1], tmp[2], tmp[15]};
            faO[mt * 5 + 3] = load_bf8(q);
        }
        faO[mt * 5 + 4] = load_bf8(tmp + 16);
    }
#define DM_SWEEP(ST, PO)                                                                                     \
    sweep_band_bf16<ST, PO>(fa, faO, sD2, (const uint32_t*)d2, a, pt, R0, seg, lam, cp, code, sCarry[wave], \
                            sDummy[wave], sK[wave])
    if ((a.w1 & 15) == 0 && a.pos) DM_SWEEP(true, true);
    else if ((a.w1 & 15) == 0) DM_SWEEP(true, false);
    else if (a.pos) DM_SWEEP(false, true);
    else DM_SWEEP(false, false);
#undef DM_SWEEP
}

__global__ __launch_bounds__(256, 2) void k_corr_pool_f32(const float* __restrict__ d1,
                                                          const float* __restrict__ d2, PoolArgs a,
                                                          float lam, float* __restrict__ cp,
                                                          uint8_t* __restrict__ code) {
    corr_f32_body(d1, d2, a, lam, cp, code, blockIdx.x);
}

__global__ __launch_bounds__(256, 2) void k_corr_pool_bf16(const uint16_t* __restrict__ d1,
                                                           const uint16_t* __restrict__ d2, PoolArgs a,
                                                           float lam, float* __restrict__ cp,
                                                           uint8_t* __restrict__ code) {
    corr_bf16_body(d1, d2, a, lam, cp, code, blockIdx.x);
}

struct CorrF32Job {
    const float *d1, *d2;
    PoolArgs a;
    float lam;
    float* cp;
    uint8_t* code;
    static __device__ void run(const CorrF32Job& j, int v) { corr_f32_body(j.d1, j.d2, j.a, j.lam, j.cp, j.code, v); }
};

struct CorrBF16Job {
    const uint16_t *d1, *d2;
    PoolArgs a;
    float lam;
    float* cp;
    uint8_t* code;
    static __device__ void run(const CorrBF16Job& j, int v) {
        corr_bf16_body(j.d1, j.d2, j.a, j.lam, j.cp, j.code, v);
    }
};

// split: allow column segments (single-pair launches; a grouped launch over
// many pairs has blocks enough without the extra step a segment costs).
PoolArgs make_pool_args(const Geom& g, int& nblocks, bool split, bool bf16) {
    PoolArgs a;
    a.natom = g.gx[0] * g.gy[0];
    a.n0x = g.gx[0];
    a.W1 = g.W1;
    a.W2 = g.W2;
    a.H2 = g.H2;
    a.h1 = g.h[1];
    a.w1 = g.w[1];
    a.pos = g.pos_corr;
    a.n_ptiles = (a.natom + (bf16 ? PT : PF) - 1) / (bf16 ? PT : PF);
    a.n_steps = (a.w1 + 15) / 16;
    // Few patches (prototype maps, small images): split the sweep into
    // column segments until about 1024 blocks exist.
    const int base = a.n_ptiles * ((a.h1 + TR - 1) / TR);
    const int want = split ? (1024 + base - 1) / base : 1;
    a.seg_steps = (a.n_steps + (want < a.n_steps ? want : a.n_steps) - 1) / (want < a.n_steps ? want : a.n_steps);
    a.n_seg = (a.n_steps + a.seg_steps - 1) / a.seg_steps;
    nblocks = base * a.n_seg;
    return a;
}

// Straightforward kernels (thread per output, direct dot products) for the
// FP64 instantiation and for a pyramid whose top is the bottom level.
template <typename T>
__device__ inline T atomic_score(const T* __restrict__ d1, const T* __restrict__ d2, const Geom& g, int b,
                                 int aa, int y, int x) {
    T acc = 0;
    for (int dy = -2; dy <= 1; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= g.H2) continue;
        for (int dx = -2; dx <= 1; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= g.W2) continue;
            const T* p = d1 + ((size_t)(2 + 4 * b + dy) * g.W1 + 2 + 4 * aa + dx) * 9;
            const T* q = d2 + ((size_t)yy * g.W2 + xx) * 9;
            for (int c = 0; c < 9; ++c) acc += p[c] * q[c];
        }
    }
    return acc / 16;
}

template <typename T>
__global__ void k_corr_top(const T* __restrict__ d1, const T* __restrict__ d2, Geom g, T lam,
                           T* __restrict__ top) {
    const size_t n = (size_t)g.gx[0] * g.gy[0] * g.H2 * g.W2;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = i % g.W2, y = (i / g.W2) % g.H2;
    const int j = i / ((size_t)g.W2 * g.H2);
    const int b = j / g.gx[0], aa = j % g.gx[0];
    T v = atomic_score(d1, d2, g, b, aa, y, x);
    top[i] = rect_pow(v > 0 ? v : T(0), lam);
}

template <typename T>
__global__ void k_corr_pool_ref(const T* __restrict__ d1, const T* __restrict__ d2, Geom g, T lam,
                                T* __restrict__ cp, uint8_t* __restrict__ code) {
    const int h1 = g.h[1], w1 = g.w[1];
    const size_t n = (size_t)g.gx[0] * g.gy[0] * h1 * w1;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = i % w1, r = (i / w1) % h1;
    const int j = i / ((size_t)w1 * h1);
    const int b = j / g.gx[0], aa = j % g.gx[0];
    T best = -1;
    int bk = 0;
    for (int my = -1; my <= 1; ++my) {
        const int y = 2 * r + my;
        if (y < 0 || y >= g.H2) continue;
        for (int mx = -1; mx <= 1; ++mx) {
            const int x = 2 * c + mx;
            if (x < 0 || x >= g.W2) continue;
            T v = atomic_score(d1, d2, g, b, aa, y, x);
            v = v > 0 ? v : T(0);
            if (v > best) {
                best = v;
                bk = 3 * (my + 1) + (mx + 1);
            }
        }
    }
    cp[i] = rect_pow(best, lam);
    code[i] = (uint8_t)bk;
}

}  // namespace

hipError_t launch_corr_pool_f32(const float* d1, const float* d2, const Geom& g, float lam, float* cp,
                                uint8_t* code, hipStream_t s) {
    int nb;
    const PoolArgs a = make_pool_args(g, nb, true, false);
    hipLaunchKernelGGL(k_corr_pool_f32, dim3(nb), dim3(256), 0, s, d1, d2, a, lam, cp, code);
    return hipGetLastError();
}

hipError_t launch_corr_pool_bf16(const uint16_t* d1, const uint16_t* d2, const Geom& g, float lam, float* cp,
                                 uint8_t* code, hipStream_t s) {
    int nb;
    const PoolArgs a = make_pool_args(g, nb, true, true);
    hipLaunchKernelGGL(k_corr_pool_bf16, dim3(nb), dim3(256), 0, s, d1, d2, a, lam, cp, code);
    return hipGetLastError();
}

JobRec corr_job(bool bf16, const void* d1, const void* d2, const Geom& g, float lam, float* cp, uint8_t* code) {
    int nb;
    const PoolArgs a = make_pool_args(g, nb, false, bf16);
    JobRec r;
    if (bf16) r.set(JK_CORR_BF16, nb, 0, CorrBF16Job{(const uint16_t*)d1, (const uint16_t*)d2, a, lam, cp, code});
    else r.set(JK_CORR_F32, nb, 0, CorrF32Job{(const float*)d1, (const float*)d2, a, lam, cp, code});
    return r;
}

hipError_t launch_group_corr(int kind, const GroupLaunch& gl, hipStream_t s) {
    if (kind == JK_CORR_BF16) return launch_grouped<CorrBF16Job, 256, 2>(gl, s);
    if (kind == JK_CORR_F32) return launch_grouped<CorrF32Job, 256, 2>(gl, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_corr_top(const T* d1, const T* d2, const Geom& g, T lam, T* top, hipStream_t s) {
    const size_t n = (size_t)g.gx[0] * g.gy[0] * g.H2 * g.W2;
    hipLaunchKernelGGL(k_corr_top<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d1, d2, g, lam, top);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_corr_pool_ref(const T* d1, const T* d2, const Geom& g, T lam, T* cp, uint8_t* code,
                                hipStream_t s) {
    const size_t n = (size_t)g.gx[0] * g.gy[0] * g.h[1] * g.w[1];
    hipLaunchKernelGGL(k_corr_pool_ref<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d1, d2, g, lam, cp,
                       code);
    return hipGetLastError();
}

template hipError_t launch_corr_top<float>(const float*, const float*, const Geom&, float, float*, hipStream_t);
template hipError_t launch_corr_top<double>(const double*, const double*, const Geom&, double, double*, hipStream_t);
template hipError_t launch_corr_pool_ref<float>(const float*, const float*, const Geom&, float, float*, uint8_t*,
                                                hipStream_t);
template hipError_t launch_corr_pool_ref<double>(const double*, const double*, const Geom&, double, double*,
                                                 uint8_t*, hipStream_t);

}  // namespace dm
