// group_c64_large.hip - instantiations of the gate-step kernels (group_impl.h) for
// float2 amplitudes and gates of 4..5 qubits; compiled as a unit of
// its own so the library builds in parallel.
#include "group_impl.h"

using namespace sts_group;

hipError_t group_c64_large_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s)
{
    switch (g.m) {
    case 4: return hist_m<float2, 4>(g, b, grid, s);
    case 5: return hist_m<float2, 5>(g, b, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c64_large_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 4: return compact_m<float2, 4>(kind, g, b, tiles, s);
    case 5: return compact_m<float2, 5>(kind, g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}

int group_c64_large_hist_capacity(int m)
{
    switch (m) {
    case 4: return hist_capacity<float2, 4>();
    case 5: return hist_capacity<float2, 5>();
    }
    return 1;
}
