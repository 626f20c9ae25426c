// Adjoint of the density solve (filled in below the forward path).
#include "sph_internal.h"

namespace sph {

hipError_t run_backward(Plan &, const int64_t *, const void *, const void *, const void *,
                        void *, void *, void *, void *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace sph
