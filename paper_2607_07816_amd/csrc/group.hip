// group.hip - dispatch of the gate-step kernels by precision and gate size
// (the kernels themselves are in group_impl.h). Gates of up to 3 qubits
// always take the LDS-tiled passes; 4-qubit gates take them when the caller
// says the side buffer has room for their larger slabs; 4- and 5-qubit gates
// otherwise take the untiled passes.
#include "kernels.h"

hipError_t group_c128_small_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s);
hipError_t group_c64_small_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s);
hipError_t group_c128_large_hist(const GateArg &g, const PassBufs &b, int grid, bool tiled, hipStream_t s);
hipError_t group_c64_large_hist(const GateArg &g, const PassBufs &b, int grid, bool tiled, hipStream_t s);
hipError_t group_c128_large_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_large_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
int group_c128_small_hist_capacity(int m);
int group_c64_small_hist_capacity(int m);
int group_c128_large_hist_capacity(int m, bool tiled);
int group_c64_large_hist_capacity(int m, bool tiled);
hipError_t group_c128_small_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_small_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c128_small_sample(const GateArg &g, const PassBufs &b, hipStream_t s);
hipError_t group_c64_small_sample(const GateArg &g, const PassBufs &b, hipStream_t s);
hipError_t group_c128_large_sample(const GateArg &g, const PassBufs &b, hipStream_t s);
hipError_t group_c64_large_sample(const GateArg &g, const PassBufs &b, hipStream_t s);
hipError_t group_c128_small_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_small_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c128_large_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_large_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c128_large_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t group_c64_large_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);

int group_hist_capacity(int prec, int m, bool tiled)
{
    if (prec == 0) return m <= 3 ? group_c128_small_hist_capacity(m) : group_c128_large_hist_capacity(m, tiled);
    return m <= 3 ? group_c64_small_hist_capacity(m) : group_c64_large_hist_capacity(m, tiled);
}

hipError_t launch_group_hist(int prec, const GateArg &g, const PassBufs &b, int grid, bool tiled, hipStream_t s)
{
    if (prec == 0)
        return g.m <= 3 ? group_c128_small_hist(g, b, grid, s) : group_c128_large_hist(g, b, grid, tiled, s);
    return g.m <= 3 ? group_c64_small_hist(g, b, grid, s) : group_c64_large_hist(g, b, grid, tiled, s);
}

hipError_t launch_group_compact(int prec, int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    if (g.m <= 3) return hipErrorInvalidValue; // small gates are always tiled
    return prec == 0 ? group_c128_large_compact(kind, g, b, tiles, s) : group_c64_large_compact(kind, g, b, tiles, s);
}

hipError_t launch_group_extract_tiles(int prec, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    if (prec == 0)
        return g.m <= 3 ? group_c128_small_extract_tiles(g, b, tiles, s) : group_c128_large_extract_tiles(g, b, tiles, s);
    return g.m <= 3 ? group_c64_small_extract_tiles(g, b, tiles, s) : group_c64_large_extract_tiles(g, b, tiles, s);
}

hipError_t launch_group_emit_tiles(int prec, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    if (prec == 0)
        return g.m <= 3 ? group_c128_small_emit_tiles(g, b, tiles, s) : group_c128_large_emit_tiles(g, b, tiles, s);
    return g.m <= 3 ? group_c64_small_emit_tiles(g, b, tiles, s) : group_c64_large_emit_tiles(g, b, tiles, s);
}

hipError_t launch_group_sample(int prec, const GateArg &g, const PassBufs &b, hipStream_t s)
{
    if (g.m < 1 || g.m > 4) return hipErrorInvalidValue; // tiled gates of 1..4 qubits only
    if (g.m == 4) return prec == 0 ? group_c128_large_sample(g, b, s) : group_c64_large_sample(g, b, s);
    return prec == 0 ? group_c128_small_sample(g, b, s) : group_c64_small_sample(g, b, s);
}
