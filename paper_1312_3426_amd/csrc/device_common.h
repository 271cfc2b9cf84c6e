// device_common.h -- D3Q19 tables, storage forms of the populations and a
// deterministic block reduction, shared by the lattice and membrane kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "oif_device.h"

namespace oif {
namespace dev {

// D3Q19 velocity set (ordering documented in include/oif.h) and weights,
// written as constexpr functions so fully unrolled loops fold them away.
__host__ __device__ constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
           : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
           : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
           : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
template <typename R>
__host__ __device__ constexpr R wt(int i) {
    return i == 0 ? R(1) / R(3) : (i <= 6 ? R(1) / R(18) : R(1) / R(36));
}

// a * b + c with one rounding
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// storage forms: S = stored type, R = arithmetic type
template <int P> struct Prec;
template <> struct Prec<PREC_FP64> { typedef double S; typedef double R; };
template <> struct Prec<PREC_FP32> { typedef float S; typedef float R; };
template <> struct Prec<PREC_FP16> { typedef uint16_t S; typedef float R; };
template <> struct Prec<PREC_BF16> { typedef uint16_t S; typedef float R; };

template <int P>
__device__ __forceinline__ typename Prec<P>::R dec(typename Prec<P>::S s, float inv);
template <>
__device__ __forceinline__ double dec<PREC_FP64>(double s, float) { return s; }
template <>
__device__ __forceinline__ float dec<PREC_FP32>(float s, float) { return s; }
template <>
__device__ __forceinline__ float dec<PREC_FP16>(uint16_t s, float inv) {
    return __half2float(__ushort_as_half(s)) * inv;
}
template <>
__device__ __forceinline__ float dec<PREC_BF16>(uint16_t s, float) {
    return __uint_as_float(((unsigned)s) << 16);
}

template <int P>
__device__ __forceinline__ typename Prec<P>::S enc(typename Prec<P>::R r, float scale);
template <>
__device__ __forceinline__ double enc<PREC_FP64>(double r, float) { return r; }
template <>
__device__ __forceinline__ float enc<PREC_FP32>(float r, float) { return r; }
template <>
__device__ __forceinline__ uint16_t enc<PREC_FP16>(float r, float scale) {
    return __half_as_ushort(__float2half_rn(r * scale));
}
template <>
__device__ __forceinline__ uint16_t enc<PREC_BF16>(float r, float) {
    // round to nearest even on the upper 16 bits; NaN stays NaN
    unsigned u = __float_as_uint(r);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Device-memory access through descriptor pointers.  Pointers read from the
// box, template and object descriptors are generic to the compiler, which then
// emits flat instructions (a 64-bit VGPR address per access, waits on both the
// LDS and the vector-memory counters).  These helpers place the access in the
// global address space as a base plus a 32-bit byte offset, so a uniform base
// stays in SGPRs and one VGPR offset serves all 19 populations of a node.
// Every array addressed this way is below 4 GiB (the context limits 19 N to
// 2^31 elements).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ T gload(const T* base, unsigned byte_off) {
    return *(gptr<const T>)((gptr<const char>)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void gstore(T* base, unsigned byte_off, T v) {
    *(gptr<T>)((gptr<char>)base + byte_off) = v;
}
template <typename T>
__device__ __forceinline__ T gload(gptr<const T> base, unsigned byte_off) {
    return *(gptr<const T>)((gptr<const char>)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void gstore(gptr<T> base, unsigned byte_off, T v) {
    *(gptr<T>)((gptr<char>)base + byte_off) = v;
}
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
    return *(gptr<const T>)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
    *(gptr<T>)p = v;
}
// Population buffers: the nodes in tiles of 64 (one wave's nodes), each tile
// holding its 19 populations one after another, 64 values each, so value
// (i, p) sits at element ((p / 64) * 19 + i) * 64 + p % 64 and a buffer holds
// 19 * ceil(N / 64) * 64 values.  A wave then reads, and mostly writes, one
// contiguous block of 19 x 64 values instead of touching 19 separate arrays.
// The context keeps the padded buffer below 2^31 elements, so p / 64 < 2^24
// and the tile product fits the 24-bit multiplier.
constexpr unsigned POP_TILE = 19u * 64u;
__device__ __forceinline__ unsigned pop_elem(int p) {
    return __umul24((unsigned)p >> 6, POP_TILE) + ((unsigned)p & 63u);
}
template <typename S>
__device__ __forceinline__ S pop_load(const S* f, int i, int p) {
    return ((gptr<const S>)f + 64 * i)[pop_elem(p)];
}
template <typename S>
__device__ __forceinline__ void pop_store(S* f, int i, int p, S v) {
    ((gptr<S>)f + 64 * i)[pop_elem(p)] = v;
}
// A wave of the lattice kernel covers exactly one tile (its blocks are whole
// multiples of 64 nodes): the tile's base is uniform and kept in SGPRs, and
// each lane addresses its own value by a 32-bit byte offset from it.
template <typename S>
__device__ __forceinline__ gptr<S> wave_tile(S* f, int p) {
    const unsigned t = __builtin_amdgcn_readfirstlane((unsigned)p >> 6);
    return (gptr<S>)f + (size_t)t * POP_TILE;
}
template <typename S>
__device__ __forceinline__ gptr<const S> wave_tile(const S* f, int p) {
    const unsigned t = __builtin_amdgcn_readfirstlane((unsigned)p >> 6);
    return (gptr<const S>)f + (size_t)t * POP_TILE;
}
// HIP's vector types are classes: load their native vector and repack
__device__ __forceinline__ int2 gld(const int2* p) {
    typedef int v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(gptr<const v2>)p;
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ int4 gld(const int4* p) {
    typedef int v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(gptr<const v4>)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gld(const double2* p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(gptr<const v2>)p;
    return make_double2(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ T gatomic_add(T* p, T v) {
    return __hip_atomic_fetch_add((gptr<T>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T gatomic_or(T* p, T v) {
    return __hip_atomic_fetch_or((gptr<T>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide FP64 sum with a fixed combination order: a butterfly inside each
// 64-lane wave (every lane ends with the same value), then the per-wave sums
// added in wave order.  Deterministic for a given block size.  `red` must hold
// one double per wave; all threads of the block must call it.
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double tot = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) tot += red[k];
    __syncthreads();
    return tot;
}

// Merge per-lane integer bounds [lo, hi] (3 axes) into the block's bbox[6]
// (lo in 0..2, hi in 3..5): reduced inside the wave by shuffles, then one LDS
// atomic per wave and axis instead of one per lane (same-address atomics
// serialise).  All lanes of each wave must call it.
__device__ inline void wave_bbox_to_block(int lo[3], int hi[3], int* bbox) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = min(lo[c], __shfl_xor(lo[c], off, 64));
            hi[c] = max(hi[c], __shfl_xor(hi[c], off, 64));
        }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            atomicMin(&bbox[c], lo[c]);
            atomicMax(&bbox[3 + c], hi[c]);
        }
}

}  // namespace dev
}  // namespace oif
