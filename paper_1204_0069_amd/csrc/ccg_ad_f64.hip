// A.D kernels (single system and batched) for FP64 matrices, one instantiation
// per padded agent count, tile width and waves per workgroup, and the symmetric
// A.D pass (k_sym, k_fin) of single FP64 systems.
#include "ccg_kernels.h"

namespace ccg {

hipError_t launch_ad_f64(int P, int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                         int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return launch_ad_prec<PREC_F64>(P, cw, nw, one, sys, items, nitems, s, e0, e1);
}

hipError_t launch_sym_f64(int P, const SymArgs& sa, const AdArgs& a, int nunits, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
    if (nunits <= 0) return hipErrorInvalidValue;
    switch (P) {
        case 1: return launch_sym_t<1>(sa, a, nunits, s, e0, e1);
        case 2: return launch_sym_t<2>(sa, a, nunits, s, e0, e1);
        case 4: return launch_sym_t<4>(sa, a, nunits, s, e0, e1);
        case 8: return launch_sym_t<8>(sa, a, nunits, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ccg
