// Instantiations of the small-system tier (k_small / k_small_batch) for each
// precision and padded agent count up to kSmallMaxP.
#include "ccg_kernels.h"

namespace ccg {

hipError_t launch_small_f64(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                            int steps, hipStream_t s) {
    return launch_small_prec<PREC_F64>(P, one, sys, items, nitems, steps, s);
}
hipError_t launch_small_f32(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                            int steps, hipStream_t s) {
    return launch_small_prec<PREC_F32>(P, one, sys, items, nitems, steps, s);
}
hipError_t launch_small_bf16(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                             int steps, hipStream_t s) {
    return launch_small_prec<PREC_BF16X2>(P, one, sys, items, nitems, steps, s);
}

}  // namespace ccg
