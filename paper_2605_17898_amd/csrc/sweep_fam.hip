// One kernel family's entry-sweep instantiations (compiled once per family
// with -DMFGP_FAM=<mfgp_family>, so the four families build in parallel).
#include "sweep_kernels.hpp"

#ifndef MFGP_FAM
#error "MFGP_FAM must be defined"
#endif

#define MFGP_CAT2(a, b) a##b
#define MFGP_CAT(a, b) MFGP_CAT2(a, b)

namespace mfgp {

hipError_t MFGP_CAT(sweep_f32_fam, MFGP_FAM)(int D, int tb, const SweepArgs& a, hipStream_t s) {
    return sweep_f32_family<MFGP_FAM>(D, tb, a, s);
}

hipError_t MFGP_CAT(sweep_f64_fam, MFGP_FAM)(int D, int tb, const SweepArgs64& a, hipStream_t s) {
    return sweep_f64_family<MFGP_FAM>(D, tb, a, s);
}

}  // namespace mfgp
