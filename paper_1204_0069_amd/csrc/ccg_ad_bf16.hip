// A.D kernels (single system and batched) for BF16 hi + lo matrices, one instantiation
// per padded agent count, tile width and waves per workgroup.
#include "ccg_kernels.h"

namespace ccg {

hipError_t launch_ad_bf16(int P, int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                         int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return launch_ad_prec<PREC_BF16X2>(P, cw, nw, one, sys, items, nitems, s, e0, e1);
}

}  // namespace ccg
