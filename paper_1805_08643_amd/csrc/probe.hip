// Data-movement probes (include/mrt_probe.h): the bytes of a lattice step
// with no arithmetic, to measure the HBM rate this part reaches for each
// access pattern the step kernels use.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/mrt_probe.h"

namespace {

thread_local std::string g_err;

lbm_status fail(const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return LBM_ERR_INVALID_ARG;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool NT, class V> __device__ inline void put(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

constexpr int kUnroll = 4;

template <bool NT>
__global__ void __launch_bounds__(256) k_probe_copy(const u32x4 *__restrict__ s, u32x4 *__restrict__ d, long long n) {
    const long long stride = (long long)gridDim.x * 256;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        u32x4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = s[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) put<NT>(d + i + u * stride, v[u]);
    }
    for (; i < n; i += stride) put<NT>(d + i, s[i]);
}

// One thread: group i of all 19 planes (plane stride `plane` groups).
template <bool NT, class V>
__global__ void __launch_bounds__(256) k_probe_stream19(const V *__restrict__ s, V *__restrict__ d, long long plane) {
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < plane; i += stride) {
        V v[19];
#pragma unroll
        for (int a = 0; a < 19; ++a) v[a] = s[a * plane + i];
#pragma unroll
        for (int a = 0; a < 19; ++a) put<NT>(d + a * plane + i, v[a]);
    }
}

struct MarchDesc {
    int nx, ny, nz, tx, ty, cz, ntx, nty, nzc, ntiles, per_xcd;
};

template <bool NT, class V>
__global__ void __launch_bounds__(256) k_probe_march19(const V *__restrict__ s, V *__restrict__ d, MarchDesc m) {
    // Tiles in contiguous ranges per XCD: block b runs tile (b mod 8) * per_xcd + b / 8.
    const int t = (int)(blockIdx.x % 8) * m.per_xcd + (int)(blockIdx.x / 8);
    if (t >= m.ntiles) return;
    const int bx = t % m.ntx, by = (t / m.ntx) % m.nty, bz = t / (m.ntx * m.nty);
    const long long plane = (long long)m.nx * m.ny, vol = plane * m.nz;
    const int z0 = bz * m.cz, z1 = min(m.nz, z0 + m.cz);
    const int ncol = m.tx * m.ty;
    for (int z = z0; z < z1; ++z) {
        for (int c = threadIdx.x; c < ncol; c += 256) {
            const int x = bx * m.tx + c % m.tx, y = by * m.ty + c / m.tx;
            if (x >= m.nx || y >= m.ny) continue;
            const long long i = z * plane + (long long)y * m.nx + x;
            V v[19];
#pragma unroll
            for (int a = 0; a < 19; ++a) v[a] = s[a * vol + i];
#pragma unroll
            for (int a = 0; a < 19; ++a) put<NT>(d + a * vol + i, v[a]);
        }
    }
}

lbm_status check_bufs(const void *s, const void *d) {
    if (!s || !d) return fail("null buffer");
    if (s == d) return fail("source and destination must differ");
    if (reinterpret_cast<uintptr_t>(s) % 256 || reinterpret_cast<uintptr_t>(d) % 256)
        return fail("buffers must be 256-byte aligned");
    return LBM_OK;
}

lbm_status launched() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_err = hipGetErrorString(e);
        return LBM_ERR_HIP;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_probe_copy(const void *src, void *dst, size_t bytes, int32_t nt, int32_t blocks, void *stream) {
    if (lbm_status s = check_bufs(src, dst)) return s;
    if (bytes == 0 || bytes % 16) return fail("bytes must be a positive multiple of 16");
    if (blocks < 0) return fail("blocks < 0");
    const dim3 grid(blocks ? blocks : 8192);
    const long long n = (long long)(bytes / 16);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nt) hipLaunchKernelGGL(k_probe_copy<true>, grid, dim3(256), 0, st, (const u32x4 *)src, (u32x4 *)dst, n);
    else hipLaunchKernelGGL(k_probe_copy<false>, grid, dim3(256), 0, st, (const u32x4 *)src, (u32x4 *)dst, n);
    return launched();
}

lbm_status lbm_probe_stream19(const void *src, void *dst, size_t plane_bytes, int32_t group_bytes, int32_t nt,
                              int32_t blocks, void *stream) {
    if (lbm_status s = check_bufs(src, dst)) return s;
    if (group_bytes != 8 && group_bytes != 16) return fail("group_bytes must be 8 or 16");
    if (plane_bytes == 0 || plane_bytes % group_bytes) return fail("plane_bytes must be a positive multiple of %d",
                                                                   group_bytes);
    if (blocks < 0) return fail("blocks < 0");
    const dim3 grid(blocks ? blocks : 8192);
    const long long plane = (long long)(plane_bytes / group_bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
#define PROBE_S19(NT, V) \
    hipLaunchKernelGGL((k_probe_stream19<NT, V>), grid, dim3(256), 0, st, (const V *)src, (V *)dst, plane)
    if (group_bytes == 8) {
        if (nt) PROBE_S19(true, u32x2);
        else PROBE_S19(false, u32x2);
    } else {
        if (nt) PROBE_S19(true, u32x4);
        else PROBE_S19(false, u32x4);
    }
#undef PROBE_S19
    return launched();
}

lbm_status lbm_probe_march19(const void *src, void *dst, int32_t nx, int32_t ny, int32_t nz, int32_t group_bytes,
                             int32_t tx, int32_t ty, int32_t cz, int32_t nt, void *stream) {
    if (lbm_status s = check_bufs(src, dst)) return s;
    if (group_bytes != 8 && group_bytes != 16) return fail("group_bytes must be 8 or 16");
    if (nx < 1 || ny < 1 || nz < 1 || tx < 1 || ty < 1 || cz < 1) return fail("sizes must be positive");
    if ((long long)tx * ty > 1024) return fail("tx * ty must be <= 1024");
    if ((__int128)nx * ny * nz * 19 >= ((__int128)1 << 40)) return fail("lattice too large");
    MarchDesc m{};
    m.nx = nx;
    m.ny = ny;
    m.nz = nz;
    m.tx = tx;
    m.ty = ty;
    m.cz = cz;
    m.ntx = (nx + tx - 1) / tx;
    m.nty = (ny + ty - 1) / ty;
    m.nzc = (nz + cz - 1) / cz;
    m.ntiles = m.ntx * m.nty * m.nzc;
    m.per_xcd = (m.ntiles + 7) / 8;
    const dim3 grid(8u * (unsigned)m.per_xcd);
    hipStream_t st = static_cast<hipStream_t>(stream);
#define PROBE_M19(NT, V) hipLaunchKernelGGL((k_probe_march19<NT, V>), grid, dim3(256), 0, st, (const V *)src, (V *)dst, m)
    if (group_bytes == 8) {
        if (nt) PROBE_M19(true, u32x2);
        else PROBE_M19(false, u32x2);
    } else {
        if (nt) PROBE_M19(true, u32x4);
        else PROBE_M19(false, u32x4);
    }
#undef PROBE_M19
    return launched();
}

const char *lbm_probe_last_error(void) { return g_err.c_str(); }

}  // extern "C"
