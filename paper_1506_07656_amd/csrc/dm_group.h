// Persistent grouped launches: one kernel launch runs the blocks of many
// jobs (one job = one stage of one image pair, with that pair's own sizes and
// buffers).  Job j owns the virtual blocks [start[j], start[j + 1]); a fixed
// grid of resident blocks walks them, block b taking b, b + grid, ...  The
// hardware deals blocks to the 8 XCDs round-robin, so every XCD gets a share
// of every job: pairs of different sizes have blocks of different cost, and
// one contiguous range of virtual blocks per XCD (which kept neighbouring
// tiles of a pair on one L2) left the XCDs with uneven work.
#pragma once

#include "dm_internal.h"

namespace dm {

// Index of the job owning virtual block v (start is increasing, start[0] = 0).
__device__ inline int group_find(const int* __restrict__ start, int njobs, int v) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Job must provide: static __device__ void run(const Job&, int block).
template <class Job, int NT, int MINB>
__global__ __launch_bounds__(NT, MINB) void k_grouped(const Job* __restrict__ jobs, const int* __restrict__ start,
                                                     int njobs, int total) {
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const int j = __builtin_amdgcn_readfirstlane(group_find(start, njobs, v));
        Job::run(jobs[j], v - start[j]);
        __syncthreads();   // LDS of one virtual block is free before the next one starts
    }
}

// Host side of one grouped launch: the job array and its block prefix live in
// device memory (written once per batch layout), grid = resident blocks.
struct GroupLaunch {
    const void* jobs;
    const int* start;
    int njobs;
    int total;   // virtual blocks
    int grid;    // resident blocks (multiple of 8)
    size_t smem; // dynamic LDS per block
};

template <class Job, int NT, int MINB>
inline hipError_t launch_grouped(const GroupLaunch& gl, hipStream_t s) {
    if (gl.njobs <= 0 || gl.total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_grouped<Job, NT, MINB>), dim3(gl.grid), dim3(NT), gl.smem, s,
                       static_cast<const Job*>(gl.jobs), gl.start, gl.njobs, gl.total);
    return hipGetLastError();
}

}  // namespace dm
