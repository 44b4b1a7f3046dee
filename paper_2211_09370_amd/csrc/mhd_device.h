// Device-side helpers shared by the gfx950 kernel sources of mhdlbm: storage traits of the
// field kinds, 32-bit-offset addressing, periodic wrap and the D3Q19 weights.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "mhd_internal.h"

namespace mhd {

// -------------------------------------------------------------------------------------------
// Storage traits
// -------------------------------------------------------------------------------------------
template <typename T>
struct St;
// cvt: stored value -> float; from: float times inverse scale -> stored value (float32 storage
// ignores the scale, which is 1 there).
template <>
struct St<float> {
    static __device__ __forceinline__ float ld(const float *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void st(float *p, int64_t i, float v) { p[i] = v; }
    static __device__ __forceinline__ float cvt(float v) { return v; }
    static __device__ __forceinline__ float val(float v, float) { return v; }
    static __device__ __forceinline__ float from(float v, float) { return v; }
};
template <>
struct St<__half> {
    static __device__ __forceinline__ float ld(const __half *p, int64_t i) { return __half2float(p[i]); }
    static __device__ __forceinline__ void st(__half *p, int64_t i, float v) { p[i] = __float2half_rn(v); }
    static __device__ __forceinline__ float cvt(__half v) { return __half2float(v); }
    static __device__ __forceinline__ float val(__half v, float scale) { return __half2float(v) * scale; }
    static __device__ __forceinline__ __half from(float v, float inv) { return __float2half_rn(v * inv); }
};
template <>
struct St<__hip_bfloat16> {
    static __device__ __forceinline__ float ld(const __hip_bfloat16 *p, int64_t i) {
        return __bfloat162float(p[i]);
    }
    static __device__ __forceinline__ void st(__hip_bfloat16 *p, int64_t i, float v) {
        p[i] = __float2bfloat16(v);
    }
    static __device__ __forceinline__ float cvt(__hip_bfloat16 v) { return __bfloat162float(v); }
    static __device__ __forceinline__ float val(__hip_bfloat16 v, float scale) { return __bfloat162float(v) * scale; }
    static __device__ __forceinline__ __hip_bfloat16 from(float v, float inv) { return __float2bfloat16(v * inv); }
};

// Element at a 32-bit byte offset from a wave-uniform base: lets the compiler use the
// scalar-base + 32-bit vector-offset addressing form instead of 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, unsigned byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_off(T *base, unsigned byte_off, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Periodic index of a neighbour one cell away (v in [-1, n]): no integer division.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Coordinates of cell k of an nx * ny * nz box in 32-bit arithmetic (boxes hold fewer than 2^31
// values per field).
__device__ __forceinline__ void cell_xyz(int64_t k, int nx, int ny, int &x, int &y, int &z) {
    const unsigned ku = (unsigned)k, q = ku / (unsigned)nx, r = q / (unsigned)ny;
    x = (int)(ku - q * (unsigned)nx);
    y = (int)(q - r * (unsigned)ny);
    z = (int)r;
}

#define W0 (1.0f / 3.0f)
#define WF (1.0f / 18.0f)
#define WE (1.0f / 36.0f)

// Supported storage mixes: all float32; rho f16 with u f16 or bf16 and b f16; all bf16;
// rho and u float32 with b float16 split.
#define MHD_KIND_F32 0
#define MHD_KIND_F16 1
#define MHD_KIND_BF16 2
#define MHD_KIND_F16_SPLIT 3  // b only, with rho and u float32 (u read by the sweeps as a float16 copy)

}  // namespace mhd
