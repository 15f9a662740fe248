// group.hip - dispatch of the gate-step kernels by precision and gate size
// (the kernels themselves are in group_impl.h).
#include "kernels.h"

hipError_t group_c128_small_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s);
hipError_t group_c128_small_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_small_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s);
hipError_t group_c64_small_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c128_large_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s);
hipError_t group_c128_large_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_large_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s);
hipError_t group_c64_large_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);

int group_c128_small_hist_capacity(int m);
int group_c64_small_hist_capacity(int m);
int group_c128_large_hist_capacity(int m);
int group_c64_large_hist_capacity(int m);

int group_hist_capacity(int prec, int m)
{
    if (prec == 0) return m <= 3 ? group_c128_small_hist_capacity(m) : group_c128_large_hist_capacity(m);
    return m <= 3 ? group_c64_small_hist_capacity(m) : group_c64_large_hist_capacity(m);
}

hipError_t launch_group_hist(int prec, const GateArg &g, const PassBufs &b, int grid, hipStream_t s)
{
    if (prec == 0) return g.m <= 3 ? group_c128_small_hist(g, b, grid, s) : group_c128_large_hist(g, b, grid, s);
    return g.m <= 3 ? group_c64_small_hist(g, b, grid, s) : group_c64_large_hist(g, b, grid, s);
}

hipError_t launch_group_compact(int prec, int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    if (prec == 0)
        return g.m <= 3 ? group_c128_small_compact(kind, g, b, tiles, s) : group_c128_large_compact(kind, g, b, tiles, s);
    return g.m <= 3 ? group_c64_small_compact(kind, g, b, tiles, s) : group_c64_large_compact(kind, g, b, tiles, s);
}

hipError_t group_c128_small_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_small_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c128_small_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_small_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);

hipError_t launch_group_extract_tiles(int prec, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    return prec == 0 ? group_c128_small_extract_tiles(g, b, tiles, s) : group_c64_small_extract_tiles(g, b, tiles, s);
}

hipError_t launch_group_emit_tiles(int prec, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    return prec == 0 ? group_c128_small_emit_tiles(g, b, tiles, s) : group_c64_small_emit_tiles(g, b, tiles, s);
}
