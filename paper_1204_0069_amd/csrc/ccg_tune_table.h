// A.D tile widths (A columns per wave) by precision, padded agent count and
// system size.  Written by `python -m paper_1204_0069_amd.tune` from timings of
// every candidate width on the GPU; the first row whose (prec, P) match and whose
// n_max >= n applies, and a size no row covers uses 2.
// Tuned on: AMD Instinct MI355X (timings of tune_ad_widths_mi355x.txt), 2026-12-03.
#pragma once

namespace ccg {

struct TuneRow {
    int prec;     // Prec
    int P;        // padded agent count
    int n_max;    // largest n of the row
    int cw;       // A columns per wave: 1, 2 or 4
};

static const TuneRow kTuneTable[] = {
    {PREC_F64, 1, 192, 2},
    {PREC_F64, 1, 384, 4},
    {PREC_F64, 1, 768, 2},
    {PREC_F64, 1, 1536, 4},
    {PREC_F64, 1, 3072, 1},
    {PREC_F64, 1, 6144, 2},
    {PREC_F64, 1, 12288, 4},
    {PREC_F64, 1, 1073741824, 2},
    {PREC_F64, 2, 192, 2},
    {PREC_F64, 2, 384, 4},
    {PREC_F64, 2, 1073741824, 2},
    {PREC_F64, 4, 192, 2},
    {PREC_F64, 4, 384, 4},
    {PREC_F64, 4, 12288, 2},
    {PREC_F64, 4, 1073741824, 4},
    {PREC_F64, 8, 384, 2},
    {PREC_F64, 8, 768, 1},
    {PREC_F64, 8, 1073741824, 2},
    {PREC_F64, 16, 384, 2},
    {PREC_F64, 16, 768, 1},
    {PREC_F64, 16, 1073741824, 2},
    {PREC_F32, 1, 192, 2},
    {PREC_F32, 1, 384, 4},
    {PREC_F32, 1, 1536, 2},
    {PREC_F32, 1, 3072, 1},
    {PREC_F32, 1, 6144, 2},
    {PREC_F32, 1, 12288, 4},
    {PREC_F32, 1, 1073741824, 2},
    {PREC_F32, 2, 192, 2},
    {PREC_F32, 2, 384, 4},
    {PREC_F32, 2, 1536, 2},
    {PREC_F32, 2, 3072, 1},
    {PREC_F32, 2, 6144, 2},
    {PREC_F32, 2, 1073741824, 4},
    {PREC_F32, 4, 192, 2},
    {PREC_F32, 4, 384, 4},
    {PREC_F32, 4, 6144, 2},
    {PREC_F32, 4, 1073741824, 4},
    {PREC_F32, 8, 192, 2},
    {PREC_F32, 8, 384, 4},
    {PREC_F32, 8, 6144, 2},
    {PREC_F32, 8, 1073741824, 4},
    {PREC_F32, 16, 1073741824, 2},
    {PREC_BF16X2, 1, 192, 2},
    {PREC_BF16X2, 1, 384, 1},
    {PREC_BF16X2, 1, 768, 4},
    {PREC_BF16X2, 1, 12288, 2},
    {PREC_BF16X2, 1, 1073741824, 1},
    {PREC_BF16X2, 2, 192, 2},
    {PREC_BF16X2, 2, 384, 4},
    {PREC_BF16X2, 2, 12288, 2},
    {PREC_BF16X2, 2, 1073741824, 4},
    {PREC_BF16X2, 4, 192, 2},
    {PREC_BF16X2, 4, 384, 1},
    {PREC_BF16X2, 4, 12288, 2},
    {PREC_BF16X2, 4, 1073741824, 4},
    {PREC_BF16X2, 8, 192, 2},
    {PREC_BF16X2, 8, 384, 1},
    {PREC_BF16X2, 8, 768, 2},
    {PREC_BF16X2, 8, 1536, 4},
    {PREC_BF16X2, 8, 6144, 2},
    {PREC_BF16X2, 8, 1073741824, 4},
    {PREC_BF16X2, 16, 192, 2},
    {PREC_BF16X2, 16, 384, 1},
    {PREC_BF16X2, 16, 1073741824, 2},
};

}  // namespace ccg
