// MFMA big contraction (placeholder until the matrix-core kernel lands).
#include "cpg_internal.h"

namespace cpg {

bool mfma_supported(int, int, int, int) { return false; }

hipError_t launch_contract_mfma(int, int, const void*, int64_t, int64_t, const FacSet<float>&, int, const Tiling&,
                                int, float*, float*, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace cpg
