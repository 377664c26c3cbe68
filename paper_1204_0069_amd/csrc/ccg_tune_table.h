// A.D tile shapes (A columns per wave, waves per workgroup) by precision, padded
// agent count and system size.  Written by `python -m paper_1204_0069_amd.tune`
// from timings of every candidate shape on the GPU; the first row whose (prec, P)
// match and whose n_max >= n applies, and a size no row covers uses 2 and 4.
// Tuned on: AMD Instinct MI355X (timings of tune_ad_widths_mi355x.txt, FP32 and BF16x2
// at P = 16 with the matrix-core shapes; FP64 P = 16 and P = 32: the matrix-core shapes
// of mfma_ad_tile_shapes_fp64.md), 2026-12-03.
#pragma once

namespace ccg {

struct TuneRow {
    int prec;     // Prec
    int P;        // padded agent count
    int n_max;    // largest n of the row
    int cw;       // A columns per wave: 1, 2 or 4
    int nw;       // waves per workgroup: 4, 8 or 16
};

static const TuneRow kTuneTable[] = {
    {PREC_F64, 1, 384, 2, 4},
    {PREC_F64, 1, 1536, 4, 4},
    {PREC_F64, 1, 6144, 2, 4},
    {PREC_F64, 1, 12288, 4, 4},
    {PREC_F64, 1, 1073741824, 2, 4},
    {PREC_F64, 2, 384, 2, 4},
    {PREC_F64, 2, 768, 4, 4},
    {PREC_F64, 2, 3072, 2, 4},
    {PREC_F64, 2, 6144, 4, 4},
    {PREC_F64, 2, 12288, 2, 4},
    {PREC_F64, 2, 1073741824, 1, 4},
    {PREC_F64, 4, 384, 2, 4},
    {PREC_F64, 4, 768, 4, 4},
    {PREC_F64, 4, 3072, 2, 4},
    {PREC_F64, 4, 6144, 4, 4},
    {PREC_F64, 4, 12288, 2, 4},
    {PREC_F64, 4, 1073741824, 4, 4},
    {PREC_F64, 8, 384, 2, 4},
    {PREC_F64, 8, 768, 2, 8},
    {PREC_F64, 8, 3072, 2, 4},
    {PREC_F64, 8, 1073741824, 2, 8},
    {PREC_F64, 16, 3072, 2, 8},
    {PREC_F64, 16, 1073741824, 4, 8},
    {PREC_F64, 32, 3072, 1, 16},
    {PREC_F64, 32, 1073741824, 2, 16},
    {PREC_F32, 1, 192, 1, 4},
    {PREC_F32, 1, 384, 2, 4},
    {PREC_F32, 1, 1536, 4, 4},
    {PREC_F32, 1, 3072, 2, 4},
    {PREC_F32, 1, 12288, 4, 4},
    {PREC_F32, 1, 1073741824, 2, 4},
    {PREC_F32, 2, 192, 1, 4},
    {PREC_F32, 2, 384, 2, 4},
    {PREC_F32, 2, 768, 4, 4},
    {PREC_F32, 2, 3072, 2, 4},
    {PREC_F32, 2, 1073741824, 4, 4},
    {PREC_F32, 4, 192, 1, 4},
    {PREC_F32, 4, 384, 2, 4},
    {PREC_F32, 4, 768, 4, 4},
    {PREC_F32, 4, 6144, 2, 4},
    {PREC_F32, 4, 1073741824, 4, 4},
    {PREC_F32, 8, 192, 1, 4},
    {PREC_F32, 8, 384, 1, 8},
    {PREC_F32, 8, 768, 2, 8},
    {PREC_F32, 8, 6144, 2, 4},
    {PREC_F32, 8, 12288, 2, 8},
    {PREC_F32, 8, 1073741824, 4, 8},
    {PREC_F32, 16, 6144, 2, 8},
    {PREC_F32, 16, 24576, 2, 16},
    {PREC_F32, 16, 1073741824, 4, 8},
    {PREC_BF16X2, 1, 192, 1, 4},
    {PREC_BF16X2, 1, 384, 2, 4},
    {PREC_BF16X2, 1, 768, 4, 4},
    {PREC_BF16X2, 1, 12288, 2, 4},
    {PREC_BF16X2, 1, 1073741824, 4, 4},
    {PREC_BF16X2, 2, 192, 1, 4},
    {PREC_BF16X2, 2, 384, 2, 4},
    {PREC_BF16X2, 2, 768, 4, 4},
    {PREC_BF16X2, 2, 12288, 2, 4},
    {PREC_BF16X2, 2, 1073741824, 4, 4},
    {PREC_BF16X2, 4, 192, 1, 4},
    {PREC_BF16X2, 4, 12288, 2, 4},
    {PREC_BF16X2, 4, 1073741824, 4, 4},
    {PREC_BF16X2, 8, 384, 1, 8},
    {PREC_BF16X2, 8, 768, 1, 4},
    {PREC_BF16X2, 8, 6144, 2, 4},
    {PREC_BF16X2, 8, 1073741824, 2, 16},
    {PREC_BF16X2, 16, 12288, 2, 8},
    {PREC_BF16X2, 16, 1073741824, 2, 16},
};

}  // namespace ccg
