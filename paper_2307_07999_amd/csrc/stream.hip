// stream.hip -- streaming kernels that measure the bandwidth a kernel of this
// library can reach on the device (the ceiling the roofline fractions of the
// field step and the push are read against): a copy, a pure read and a pure
// write of large buffers in 16-byte accesses, in a few access patterns.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/glasma.h"

namespace {

thread_local std::string g_err;

gl_status sfail(gl_status s, const std::string &m) {
    g_err = m;
    return s;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ u32x4 ld(const u32x4 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(u32x4 *p, u32x4 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// kind 0 copy, 1 read (the xor of everything, one word per workgroup written),
// 2 write (a fill).  UNROLL 16-byte vectors per lane and pass, loads issued
// before the stores.  Grid-stride over n vectors; BLOCKED: each workgroup
// walks one contiguous share of the buffer instead of interleaving with the
// others.
template <int KIND, bool NT, int UNROLL, bool BLOCKED>
__global__ void __launch_bounds__(256)
k_stream(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, int64_t n) {
    const int64_t per_pass = (int64_t)256 * UNROLL;
    int64_t begin, end, step, i0;
    if (BLOCKED) {
        const int64_t share = (n + gridDim.x - 1) / gridDim.x;
        begin = (int64_t)blockIdx.x * share;
        end = begin + share < n ? begin + share : n;
        step = per_pass;
        i0 = begin + threadIdx.x;
    } else {
        begin = 0;
        end = n;
        step = per_pass * gridDim.x;
        i0 = (int64_t)blockIdx.x * per_pass + threadIdx.x;
    }
    u32x4 acc = {0u, 0u, 0u, 0u};
    const u32x4 fill = {0x3f800000u, 0u, 0x3f800000u, 0u};
    for (int64_t i = i0; i < end; i += step) {
        u32x4 v[UNROLL];
        if (KIND != 2) {
#pragma unroll
            for (int u = 0; u < UNROLL; u++) {
                const int64_t k = i + (int64_t)u * 256;
                v[u] = k < end ? ld<NT>(src + k) : u32x4{0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; u++) {
            const int64_t k = i + (int64_t)u * 256;
            if (k < end) {
                if (KIND == 0) st<NT>(dst + k, v[u]);
                else if (KIND == 2) st<NT>(dst + k, fill);
                else acc ^= v[u];
            }
        }
    }
    (void)begin;
    if (KIND == 1) {
        // keep the loads live: the workgroup's xor of everything it read, one
        // 16-byte word per workgroup
        __shared__ unsigned red[256];
        red[threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned x = 0;
            for (int t = 0; t < 256; t++) x ^= red[t];
            dst[blockIdx.x] = u32x4{x, 0u, 0u, 0u};
        }
    }
}

template <int KIND>
hipError_t launch_variant(int variant, const u32x4 *src, u32x4 *dst, int64_t n, int blocks, hipStream_t st) {
    dim3 g(blocks), b(256);
    switch (variant) {
        case 0: hipLaunchKernelGGL((k_stream<KIND, false, 1, false>), g, b, 0, st, src, dst, n); break;
        case 1: hipLaunchKernelGGL((k_stream<KIND, false, 4, false>), g, b, 0, st, src, dst, n); break;
        case 2: hipLaunchKernelGGL((k_stream<KIND, true, 4, false>), g, b, 0, st, src, dst, n); break;
        case 3: hipLaunchKernelGGL((k_stream<KIND, false, 4, true>), g, b, 0, st, src, dst, n); break;
        case 4: hipLaunchKernelGGL((k_stream<KIND, true, 4, true>), g, b, 0, st, src, dst, n); break;
        case 5: hipLaunchKernelGGL((k_stream<KIND, true, 8, false>), g, b, 0, st, src, dst, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

gl_status gl_stream_probe(int32_t kind, int32_t variant, int32_t blocks, const void *src, void *dst, size_t bytes,
                          size_t dst_bytes, int32_t reps, void *stream, double *ms_avg) {
    if (!ms_avg || reps < 1 || kind < 0 || kind > 2 || variant < 0 || variant >= GL_STREAM_VARIANTS || blocks < 1)
        return sfail(GL_EINVAL, "bad argument");
    if ((kind != 2 && !src) || !dst || bytes < 16 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return sfail(GL_EINVAL, "buffers must be non-null, 16-byte aligned, and bytes a multiple of 16");
    if (dst_bytes < (kind == 1 ? (size_t)blocks * 16 : bytes))
        return sfail(GL_EINVAL, "dst too small (bytes for copy and write, 16 per workgroup for read)");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)(bytes / 16);
    auto launch = [&]() -> hipError_t {
        const u32x4 *s = (const u32x4 *)src;
        u32x4 *d = (u32x4 *)dst;
        if (kind == 0) return launch_variant<0>(variant, s, d, n, blocks, st);
        if (kind == 1) return launch_variant<1>(variant, s, d, n, blocks, st);
        return launch_variant<2>(variant, s, d, n, blocks, st);
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return sfail(GL_EDEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return sfail(GL_EDEVICE, "hipEventCreate failed");
    }
    gl_status s = GL_OK;
    float ms = 0.f;
    hipError_t e = launch();   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; r++) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) s = sfail(GL_EDEVICE, std::string("stream probe: ") + hipGetErrorString(e));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!s) *ms_avg = (double)ms / reps;
    return s;
}

const char *gl_stream_last_error(void) { return g_err.c_str(); }

}  // extern "C"
