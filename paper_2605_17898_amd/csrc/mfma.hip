// BF16-MFMA tile products: placeholder until the MFMA kernels land.
#include "internal.hpp"

namespace mfgp {

bool precision_supported(int p) { return p == MFGP_FP32; }

size_t mfma_scratch_bytes(int64_t, int64_t, int, int) { return 0; }

hipError_t apply_mfma(const Operator&, const float*, int64_t, const float*, int, float*, bool,
                      const float*, int, void*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace mfgp
