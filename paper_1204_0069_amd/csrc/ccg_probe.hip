// Read-stream ceiling of the A.D traffic shape (a measurement aid, not in the paper).
//
// k_stream reads an n x n FP64 matrix stored column-major with lda = n, `cols`
// whole columns (one contiguous chunk of cols * n doubles) per workgroup of WG
// threads, with 16-byte non-temporal loads, and adds it up.  With an n x dcols block D it also
// reads the whole of D in every workgroup, spread over its chunk, as the A.D tile
// kernel does with the direction block.  With `stagger`, workgroup b starts its
// chunk at step (13 b) mod steps and wraps around, as the A.D kernel staggers its
// tiles.  It does no other work, so its time is the floor that the memory system
// sets for that pattern of traffic.  k_grid_stride (stagger = 2) reads the same
// bytes with no column ownership at all: on every pass the workgroups together
// read one contiguous span of nwg * WG * 4 vectors, and the next pass starts where
// it ended, the plain streaming ceiling of the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ccg_host.h"

namespace ccg {
namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int WG>
__global__ __launch_bounds__(WG) void k_stream(const dvec2* __restrict__ a, int64_t chunk,
                                               const dvec2* __restrict__ d, int64_t dlen, int stagger,
                                               double* out) {
    constexpr int U = 4;
    const dvec2* p = a + (int64_t)blockIdx.x * chunk;
    const int64_t steps = (chunk + WG * U - 1) / (WG * U);
    const int64_t dstep = d ? (dlen + steps - 1) / steps : 0;
    double s = 0.0;
    const int64_t k0 = stagger ? (13 * (int64_t)blockIdx.x) % steps : 0;
    for (int64_t kk = 0; kk < steps; ++kk) {
        const int64_t k = (k0 + kk) % steps;
        const int64_t i = threadIdx.x + k * WG * U;
        dvec2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = (i + u * WG < chunk) ? __builtin_nontemporal_load(&p[i + u * WG]) : dvec2{0.0, 0.0};
        for (int64_t j = k * dstep + threadIdx.x; j < (k + 1) * dstep && j < dlen; j += WG) {
            const dvec2 w = d[j];
            s += w.x * w.y;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u].x + v[u].y;
    }
    __shared__ double red[WG];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

template <int WG>
__global__ __launch_bounds__(WG) void k_grid_stride(const dvec2* __restrict__ a, int64_t total, double* out) {
    constexpr int U = 4;
    const int64_t span = (int64_t)gridDim.x * WG * U;
    double s = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * WG * U + threadIdx.x; base < total; base += span) {
        dvec2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = (base + u * WG < total) ? __builtin_nontemporal_load(&a[base + u * WG]) : dvec2{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u].x + v[u].y;
    }
    __shared__ double red[WG];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace
}  // namespace ccg

using namespace ccg;
using namespace ccg::host;

extern "C" ccg_status ccg_stream_probe(ccg_ctx* c, int n, int cols, int dcols, int stagger, int waves,
                                       int reps, double* us) {
    return guarded(c, [&]() -> ccg_status {
        if (n < 2 || n % 2 || cols < 1 || n % cols || dcols < 0 || dcols > kMaxP || reps < 1 || !us ||
            (waves != 4 && waves != 8 && waves != 16) || stagger < 0 || stagger > 2 || (stagger == 2 && dcols))
            throw CcgError{CCG_ERR_ARG,
                           "bad probe argument (n even, cols dividing n, 0 <= dcols <= 16, waves 4, 8 or 16, "
                           "stagger 0, 1 or 2 (grid-stride, no D))"};
        const size_t elems = (size_t)n * n;
        const int nwg = n / cols;
        void* buf = nullptr;
        const size_t dbytes = sizeof(double) * (size_t)n * (dcols > 0 ? dcols : 1);
        const size_t bytes = sizeof(double) * elems + dbytes + sizeof(double) * (size_t)nwg + 512;
        if (hipMalloc(&buf, bytes) != hipSuccess) throw CcgError{CCG_ERR_NOMEM, "probe allocation failed"};
        struct Free {
            void* p;
            ~Free() { (void)hipFree(p); }
        } fb{buf};
        char* base = static_cast<char*>(buf);
        const dvec2* a = reinterpret_cast<const dvec2*>(base);
        const size_t doff = round_up((int64_t)(sizeof(double) * elems), 256);
        const dvec2* d = dcols > 0 ? reinterpret_cast<const dvec2*>(base + doff) : nullptr;
        double* out = reinterpret_cast<double*>(base + round_up((int64_t)(doff + dbytes), 256));
        HIP_OK(hipMemsetAsync(buf, 0, bytes, c->stream));
        const int64_t chunk = (int64_t)cols * n / 2;      // 16-byte vectors per workgroup
        const int64_t dlen = (int64_t)n * dcols / 2;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        std::vector<float> t;
        ccg_status st = CCG_OK;
        for (int r = 0; r < reps + 2 && st == CCG_OK; ++r) {
            if (hipEventRecord(e0, c->stream) != hipSuccess) { st = CCG_ERR_DEVICE; break; }
            const int sg = stagger ? 1 : 0;
            if (stagger == 2) {
                const int64_t total = (int64_t)elems / 2;
                if (waves == 4)
                    hipLaunchKernelGGL(k_grid_stride<256>, dim3(nwg), dim3(256), 0, c->stream, a, total, out);
                else if (waves == 8)
                    hipLaunchKernelGGL(k_grid_stride<512>, dim3(nwg), dim3(512), 0, c->stream, a, total, out);
                else
                    hipLaunchKernelGGL(k_grid_stride<1024>, dim3(nwg), dim3(1024), 0, c->stream, a, total, out);
            } else if (waves == 4)
                hipLaunchKernelGGL(k_stream<256>, dim3(nwg), dim3(256), 0, c->stream, a, chunk, d, dlen, sg, out);
            else if (waves == 8)
                hipLaunchKernelGGL(k_stream<512>, dim3(nwg), dim3(512), 0, c->stream, a, chunk, d, dlen, sg, out);
            else
                hipLaunchKernelGGL(k_stream<1024>, dim3(nwg), dim3(1024), 0, c->stream, a, chunk, d, dlen, sg, out);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, c->stream) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess) {
                st = CCG_ERR_DEVICE;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r >= 2) t.push_back(ms);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != CCG_OK) throw CcgError{st, "probe launch failed"};
        std::sort(t.begin(), t.end());
        *us = t[t.size() / 2] * 1e3;
        return CCG_OK;
    });
}
