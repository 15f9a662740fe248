// group_c64_small.hip - instantiations of the gate-step kernels (group_impl.h)
// for float2 amplitudes and gates of 0..3 qubits; compiled as a unit of its
// own so the library builds in parallel.
#include "group_impl.h"

using namespace sts_group;

hipError_t group_c64_small_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s)
{
    switch (g.m) {
    case 0: return hist_m<float2, 0, true>(g, b, grid, s);
    case 1: return hist_m<float2, 1, true>(g, b, grid, s);
    case 2: return hist_m<float2, 2, true>(g, b, grid, s);
    case 3: return hist_m<float2, 3, true>(g, b, grid, s);
    }
    return hipErrorInvalidValue;
}

int group_c64_small_hist_capacity(int m)
{
    switch (m) {
    case 0: return hist_capacity<float2, 0, true>();
    case 1: return hist_capacity<float2, 1, true>();
    case 2: return hist_capacity<float2, 2, true>();
    case 3: return hist_capacity<float2, 3, true>();
    }
    return 1;
}

hipError_t group_c64_small_extract_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 0: return extract_tiles_m<float2, 0>(g, b, tiles, s);
    case 1: return extract_tiles_m<float2, 1>(g, b, tiles, s);
    case 2: return extract_tiles_m<float2, 2>(g, b, tiles, s);
    case 3: return extract_tiles_m<float2, 3>(g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c64_small_emit_tiles(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 0: return emit_tiles_m<float2, 0>(g, b, tiles, s);
    case 1: return emit_tiles_m<float2, 1>(g, b, tiles, s);
    case 2: return emit_tiles_m<float2, 2>(g, b, tiles, s);
    case 3: return emit_tiles_m<float2, 3>(g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c64_small_sample(const GateArg &g, const PassBufs &b, hipStream_t s)
{
    switch (g.m) {
    case 1: return sample_m<float2, 1>(g, b, s);
    case 2: return sample_m<float2, 2>(g, b, s);
    case 3: return sample_m<float2, 3>(g, b, s);
    }
    return hipErrorInvalidValue;
}
