// Measurement helpers: the streaming bandwidth a plain read-and-write kernel
// reaches on this GPU, at a given element size, the practical memory ceiling
// the translation kernels are compared with (they read each level's state
// once and write the next level's once, with the same element sizes); and
// the FP64 matrix-core rate sustained by independent 16 x 16 x 4 products,
// the practical ceiling of the matrix-core direct sums.
#include "bfsft_impl.h"

#include <algorithm>
#include <string>
#include <vector>

namespace bfsft {

namespace {

// dst[i] = src[i] over n elements of the translation's access width: each
// work-group copies 4 x 256 consecutive elements, each thread four of them
// 256 apart (every access instruction of a wave is one contiguous range),
// with its four loads issued before its stores
template <typename T>
__global__ __launch_bounds__(256) void k_stream_copy(const T *__restrict__ src, T *__restrict__ dst, int64_t n)
{
    const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    T v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (i0 + 256 * j < n) v[j] = src[i0 + 256 * j];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (i0 + 256 * j < n) dst[i0 + 256 * j] = v[j];
}

template <typename T> void launch_copy(const void *src, void *dst, int64_t bytes, unsigned grid, hipStream_t s)
{
    k_stream_copy<T><<<grid, 256, 0, s>>>((const T *)src, (T *)dst, bytes / (int64_t)sizeof(T));
}

typedef double dx4 __attribute__((ext_vector_type(4)));
constexpr int kRateChains = 12;  // independent accumulators per wave, as in the direct sums

// `iters` rounds of 12 independent v_mfma_f64_16x16x4f64 per wave; one wave
// per SIMD per work-group of 256 threads.  Operands come from `in` (64 + 64
// values) so that nothing folds; each thread writes one sum to out.
__global__ __launch_bounds__(256) void k_mfma_f64_rate(const double *__restrict__ in, double *__restrict__ out,
                                                       int iters)
{
    double a = in[threadIdx.x & 63];
    const double b = in[64 + (threadIdx.x & 63)];
    dx4 acc[kRateChains];
#pragma unroll
    for (int k = 0; k < kRateChains; ++k) acc[k] = dx4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kRateChains; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
        a = fma(a, 0.5, 0.25);  // stays near 0.5
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kRateChains; ++k) sum += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

}  // namespace

}  // namespace bfsft

using namespace bfsft;

extern "C" int bfsft_copy_rate(int elem_bytes, int64_t bytes, int reps, void *stream, double *gbps)
{
    if (!gbps || reps < 1 || bytes < (1 << 20) || bytes > ((int64_t)1 << 34) ||
        (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) || bytes % elem_bytes) {
        set_last_error("bfsft_copy_rate: elem_bytes must be 4, 8 or 16, bytes a multiple of it in "
                       "[2^20, 2^34], reps >= 1, gbps not NULL");
        return BFSFT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BFSFT_OK;
    auto fail = [&](hipError_t e, int status) {
        set_last_error(std::string("bfsft_copy_rate: ") + hipGetErrorString(e));
        rc = status;
    };
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e != hipSuccess) {
        fail(e, BFSFT_ENOMEM);
    } else {
        const int64_t n = bytes / elem_bytes;
        // one work-group per 1024 elements (at most 2^22 of them: 2^34 bytes of 4-byte elements)
        const unsigned grid = (unsigned)((n + 1023) / 1024);
        auto launch = [&] {
            if (elem_bytes == 4) launch_copy<float>(a, b, bytes, grid, s);
            else if (elem_bytes == 8) launch_copy<float2>(a, b, bytes, grid, s);
            else launch_copy<float4>(a, b, bytes, grid, s);
        };
        e = hipMemsetAsync(a, 0, bytes, s);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) {
            launch();  // untimed
            e = hipEventRecord(e0, s);
        }
        if (e == hipSuccess) {
            for (int r = 0; r < reps; ++r) launch();
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess)
            fail(e, BFSFT_EDEVICE);
        else
            *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return rc;
}

extern "C" int bfsft_mfma_f64_rate(int waves_per_simd, int iters, void *stream, double *tflops)
{
    if (!tflops || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || iters > (1 << 20)) {
        set_last_error("bfsft_mfma_f64_rate: waves_per_simd in [1, 8], iters in [1, 2^20], tflops not NULL");
        return BFSFT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || ncu < 1) {
        set_last_error(std::string("bfsft_mfma_f64_rate: ") + hipGetErrorString(e));
        return BFSFT_EDEVICE;
    }
    const int blocks = ncu * waves_per_simd;
    double *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BFSFT_OK;
    e = hipMalloc(&buf, sizeof(double) * (128 + (size_t)blocks * 256));
    if (e != hipSuccess) {
        set_last_error(std::string("bfsft_mfma_f64_rate: ") + hipGetErrorString(e));
        return BFSFT_ENOMEM;
    }
    std::vector<double> ones(128, 1.0);
    e = hipMemcpyAsync(buf, ones.data(), sizeof(double) * 128, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        k_mfma_f64_rate<<<blocks, 256, 0, s>>>(buf, buf + 128, std::min(iters, 64));  // untimed
        e = hipEventRecord(e0, s);
    }
    if (e == hipSuccess) {
        k_mfma_f64_rate<<<blocks, 256, 0, s>>>(buf, buf + 128, iters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
        set_last_error(std::string("bfsft_mfma_f64_rate: ") + hipGetErrorString(e));
        rc = BFSFT_EDEVICE;
    } else {
        // 4 waves per work-group, 12 MFMAs of 16 x 16 x 4 x 2 flops per round
        *tflops = (double)blocks * 4.0 * iters * kRateChains * 2048.0 / (ms * 1e-3) / 1e12;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return rc;
}
