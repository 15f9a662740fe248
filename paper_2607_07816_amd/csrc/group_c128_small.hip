// group_c128_small.hip - instantiations of the gate-step kernels (group_impl.h) for
// double2 amplitudes and gates of 0..3 qubits; compiled as a unit of
// its own so the library builds in parallel.
#include "group_impl.h"

using namespace sts_group;

hipError_t group_c128_small_hist(const GateArg &g, const PassBufs &b, int grid, hipStream_t s)
{
    switch (g.m) {
    case 0: return hist_m<double2, 0>(g, b, grid, s);
    case 1: return hist_m<double2, 1>(g, b, grid, s);
    case 2: return hist_m<double2, 2>(g, b, grid, s);
    case 3: return hist_m<double2, 3>(g, b, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t group_c128_small_compact(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    switch (g.m) {
    case 0: return compact_m<double2, 0>(kind, g, b, tiles, s);
    case 1: return compact_m<double2, 1>(kind, g, b, tiles, s);
    case 2: return compact_m<double2, 2>(kind, g, b, tiles, s);
    case 3: return compact_m<double2, 3>(kind, g, b, tiles, s);
    }
    return hipErrorInvalidValue;
}
