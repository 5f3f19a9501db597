"""Host-side model of the index arithmetic of the backtracking kernels
(k_backtrack.hip): the bottom step's cell-table window and table index, and
the streaming form's candidate ring, for every argmax code 0..8 at the first
and last rows and columns of every band and tile, on the I' sizes the GPU
tests and the benchmark use.

A tuple at pooled position (ry, rx) with code k = 3(m_y + 1) + (m_x + 1)
lands on target pixel (2 ry + m_y, 2 rx + m_x).  The forward pool never picks
a window position outside I', so a code that the pyramid can produce keeps
that pixel inside I'; the kernels rely on this and check nothing more.  The
model shows that every such code stays inside the LDS window and the cell
table, and that a code the pool cannot produce at the border (a pixel at -1
or past the last row or column) leaves the cell table: the final flush would
write outside it.
"""
import itertools

import pytest

# Constants of the streaming form (k_backtrack.hip).
BT_COLS = 64                     # lanes per wave, width of the candidate ring
BT_RING = 8                      # candidate rows in the ring
BT_MAX_TR = 64                   # tallest band
NCX = BT_COLS // 2 + 2           # cell-window columns of the streaming form
SCELL_STREAM = (BT_MAX_TR // 2 + 2) * NCX

# I' sizes of the tests (c1, c2, c3, odd, narrow, wide540/544, batch recipe
# extremes and odd crops).
TARGETS = [(64, 64), (256, 192), (512, 256), (300, 156), (200, 148), (540, 72), (544, 72), (128, 96), (621, 188),
           (101, 128), (19, 41), (5, 3), (3, 2), (1, 1), (157, 99)]


def pixel(ry, rx, k):
    return 2 * ry + k // 3 - 1, 2 * rx + k % 3 - 1


def valid(ry, rx, k, H2, W2):
    y, x = pixel(ry, rx, k)
    return 0 <= y < H2 and 0 <= x < W2


def border_positions(R0, R1, C0, C1):
    rows = sorted({R0, R0 + 1, R1 - 2, R1 - 1} & set(range(R0, R1)))
    cols = sorted({C0, C0 + 1, C1 - 2, C1 - 1} & set(range(C0, C1)))
    return itertools.product(rows, cols)


def check_bottom_window(H2, W2, R0, R1, C0, C1, ncy, ncx, lds_cells):
    """Every tuple of the band/tile [R0, R1) x [C0, C1) of the pooled level-0
    grid: its cell is inside the window and the table.  Returns the number of
    invalid border codes whose cell leaves the table."""
    cyb, cxb = (2 * R0 - 1) >> 2, (2 * C0 - 1) >> 2       # floor division, as the kernel's >> 2
    ch, cw = (H2 + 3) // 4, (W2 + 3) // 4
    escapes = 0
    for ry, rx in border_positions(R0, R1, C0, C1):
        for k in range(9):
            y, x = pixel(ry, rx, k)
            wy, wx = (y >> 2) - cyb, (x >> 2) - cxb
            in_window = 0 <= wy < ncy and 0 <= wx < ncx and wy * ncx + wx < lds_cells
            in_table = 0 <= (y >> 2) < ch and 0 <= (x >> 2) < cw
            if valid(ry, rx, k, H2, W2):
                assert in_window, (H2, W2, R0, C0, ry, rx, k)
                assert in_table, (H2, W2, R0, C0, ry, rx, k)
            elif in_window and not in_table:
                escapes += 1
    return escapes


@pytest.mark.parametrize("W2,H2", TARGETS)
@pytest.mark.parametrize("tile", [60, 64])
def test_streaming_bottom_cell_window(W2, H2, tile):
    h, w = (H2 + 1) // 2, (W2 + 1) // 2      # pooled level-0 grid: the child maps of level 1
    escapes = 0
    for tr in (2, 8, 16, 32, 64):
        TR = ((h + 1) & ~1) if h < tr else tr
        ncy = TR // 2 + 2
        assert ncy * NCX <= SCELL_STREAM
        for R0 in range(0, h, TR):
            for C0 in range(0, w, tile):
                escapes += check_bottom_window(H2, W2, R0, min(R0 + TR, h), C0, min(C0 + tile, w), ncy, NCX,
                                               SCELL_STREAM)
    # a code naming a pixel outside I' at the border would be flushed outside the table
    if H2 > 1 and W2 > 1:
        assert escapes > 0


@pytest.mark.parametrize("W2,H2", TARGETS)
def test_tiled_bottom_cell_window(W2, H2):
    h, w = (H2 + 1) // 2, (W2 + 1) // 2
    TC = w if w < 128 else 128
    TR = max(1, min(1024 // TC, h))
    ncy, ncx = TR // 2 + 2, TC // 2 + 2
    for R0 in range(0, h, TR):
        for C0 in range(0, w, TC):
            check_bottom_window(H2, W2, R0, min(R0 + TR, h), C0, min(C0 + TC, w), ncy, ncx, ncy * ncx)


@pytest.mark.parametrize("W2,H2", TARGETS)
@pytest.mark.parametrize("tile", [60, 64])
def test_streaming_ring_rows(W2, H2, tile):
    """At parent row rp a scattered candidate lands on child rows
    2 rp - 2 .. 2 rp + 2, and rows 2 rp - 2, 2 rp - 1 are taken out: the five
    live rows have distinct ring slots, no later parent row reaches a row
    already taken out, and every column a lane scatters to inside the tile is
    a ring column."""
    h, w = (H2 + 1) // 2, (W2 + 1) // 2           # child pooled grid (level 0) and level-1 maps
    hu, wu = (h + 1) // 2, (w + 1) // 2           # parent U grid
    for tr in (2, 8, 64):
        TR = ((h + 1) & ~1) if h < tr else tr
        for R0 in range(0, h, TR):
            R1 = min(R0 + TR, h)
            rp0, rp1 = (R0 - 1) >> 1, ((R1 - 1) >> 1) + 1
            for rp in range(rp0, rp1 + 1):
                live = set(range(2 * rp - 2, 2 * rp + 3))
                assert len({r & (BT_RING - 1) for r in live}) == len(live)
                for taken in (2 * rp - 2, 2 * rp - 1):
                    assert all(not (2 * q - 2 <= taken <= 2 * q + 2) for q in range(rp + 1, rp1 + 2))
            for C0 in range(0, w, tile):
                Cend = min(C0 + tile, w)
                for t in range(64):
                    ux = (C0 >> 1) - 1 + ((t & 31) if tile == 60 else t)
                    if not ((tile == 60 or t < tile // 2 + 2) and 0 <= ux < wu):
                        continue
                    for k, sx in itertools.product(range(9), (-1, 1)):
                        if not (0 <= 2 * ux + k % 3 - 1 < w):
                            continue
                        rxx = 2 * ux + k % 3 - 1 + sx
                        if C0 <= rxx < Cend:
                            assert 0 <= rxx - C0 < BT_COLS
