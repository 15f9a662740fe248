// group_c64_large.hip - instantiations of the gate-step kernels (group_impl.h)
// for float2 amplitudes and gates of 4..5 qubits; compiled as a unit of its
// own so the library builds in parallel.
#include "group_impl.h"

using namespace sts_group;

hipError_t group_c64_large_hist(const GateArg &g, const PassBufs &b, int grid, bool tiled, hipStream_t s)
{
    if (g.m == 4 && tiled) return hist_m<float2, 4, true>(g, b, grid, s);
    switch (g.m) {
    case 4: return hist_m<float2, 4, false>(g, b, grid, s);
    case 5: return hist_m<float2, 5, false>(g, b, grid, s);
    }
    return hipErrorInvalidValue;
}

int group_c64_large_hist_capacity(int m, bool tiled)
{
    if (m == 4 && tiled) return hist_capacity<float2, 4, true>();
    switch (m) {
    case 4: return hist_capacity<float2, 4, false>();
    case 5: return hist_capacity<float2, 5, false>();
    }
    return 1;
}

hipError_t group_c64_large_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 4: return compact_m<float2, 4>(kind, g, b, tiles, s);
    case 5: return compact_m<float2, 5>(kind, g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c64_large_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 4: return extract_tiles_m<float2, 4>(g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c64_large_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 4: return emit_tiles_m<float2, 4>(g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c64_large_sample(const GateArg &g, const PassBufs &b, hipStream_t s)
{
    switch (g.m) {
    case 4: return sample_m<float2, 4>(g, b, s);
    }
    return hipErrorInvalidValue;
}
