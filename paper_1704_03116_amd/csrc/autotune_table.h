// Block partition table of dope_autotune, written by paper_1704_03116_amd/tune.py from an MI355X sweep
// (whole-solve throughput of serving-style images per stencil and size; the measurements are kept in
// profiles/autotune_sweep.json).  Row: ndim, connectivity, largest shorter side, block edge B, overlap o.
#pragma once

namespace dope {

struct TuneRow {
    int ndim, conn, max_short_side, block, overlap;
};

constexpr TuneRow TUNE_TABLE[] = {
    {2, 4, 181, 16, 1},
    {2, 4, 362, 16, 2},
    {2, 4, 724, 16, 2},
    {2, 4, 1448, 32, 1},
    {2, 4, 2147483647, 32, 1},
    {2, 8, 181, 32, 2},
    {2, 8, 362, 16, 1},
    {2, 8, 724, 16, 2},
    {2, 8, 1448, 32, 1},
    {2, 8, 2147483647, 32, 1},
    {2, 24, 181, 16, 4},
    {2, 24, 362, 16, 4},
    {2, 24, 724, 16, 2},
    {2, 24, 2147483647, 16, 2},
    {2, 48, 181, 16, 2},
    {2, 48, 362, 16, 2},
    {2, 48, 2147483647, 16, 2},
    {2, 80, 181, 16, 2},
    {2, 80, 362, 16, 2},
    {2, 80, 2147483647, 16, 2},
    {3, 6, 22, 12, 2},
    {3, 6, 39, 8, 1},
    {3, 6, 2147483647, 8, 1},
    {3, 32, 22, 6, 1},
    {3, 32, 2147483647, 10, 2},
    {3, 122, 2147483647, 6, 2},
};

}  // namespace dope
