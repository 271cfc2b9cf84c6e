// lb_kernels.hip -- lattice kernels of the coupled step (paper, Section
// "Method": the D3Q19 propagation/collision update with an external force
// term, eq. lbequation, and the moment definitions of density and velocity).
//
//   lb_kernel   one lattice node per thread: decode the 19 stored deviations,
//               BGK collision with Guo forcing (force density g + G, the
//               step's G read only where the node's mask bit is set, the bit
//               cleared; the membrane kernel zeroes G in the next step), push the
//               19 post-collision values to the neighbours (halfway
//               bounce-back at z walls), encode.  HBM bound: every node reads
//               and writes 19 stored values once, 2 x 19 x sizeof(storage)
//               bytes per node; the force read adds 24 bytes only at nodes
//               touched by the spreading.
//   diag_*      FP64 sums of mass and momentum and a non-finite watchdog,
//               two passes with a fixed summation order (deterministic).
//   *_to_*      conversions between the storage form and canonical FP64 fields.
#include "lb_device.h"

namespace oif {
namespace {

using namespace dev;

// the lattice update of one node: lb_device.h

template <int P, bool OBST, bool ALL, bool MRT, bool NT>
__global__ void __launch_bounds__(1024)
lb_kernel(const BoxDev* __restrict__ boxes, const int2* __restrict__ work, int nblocks, int parity,
          int remap, int mode) {
    int bid = blockIdx.x;
    if (remap) {
        // workgroups are dispatched round-robin over the 8 XCDs; give each XCD
        // a contiguous range of lattice blocks so neighbouring planes share an L2
        const int full = nblocks & ~7;
        if (bid < full) bid = (bid & 7) * (full >> 3) + (bid >> 3);
    }
    int box = 0, blk = bid;
    if (work) {
        const int2 w = work[bid];
        box = w.x;
        blk = w.y;
    }
    lb_node<P, OBST, ALL, MRT, NT>(boxes + box, blk * (int)blockDim.x + (int)threadIdx.x, parity, mode);
}

template <int P>
__global__ void __launch_bounds__(1024)
diag_lattice_kernel(const BoxDev* __restrict__ B, int parity, double* __restrict__ part) {
    typedef typename Prec<P>::S S;
    __shared__ double red[16];
    const S* __restrict__ src = (const S*)B->f[parity];
    const int N = B->N;
    const float inv = B->st_inv;
    double dm = 0, jx = 0, jy = 0, jz = 0, bad = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        double d[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            d[i] = (double)dec<P>(pop_load(src, i, p), inv);
            if (!isfinite(d[i])) bad = 1.0;
        }
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            dm += d[i];
            jx += cx(i) * d[i];
            jy += cy(i) * d[i];
            jz += cz(i) * d[i];
        }
    }
    const double s0 = block_sum(dm, red), s1 = block_sum(jx, red), s2 = block_sum(jy, red),
                 s3 = block_sum(jz, red), s4 = block_sum(bad, red);
    if (threadIdx.x == 0) {
        double* o = part + 5 * blockIdx.x;
        o[0] = s0; o[1] = s1; o[2] = s2; o[3] = s3; o[4] = s4;
    }
}

// The five sums of the lattice blocks' partials and of the objects' partials
// in a fixed order (thread t adds partials t, t + 256, ... in turn, then a fixed
// tree over the 256 threads): the same bits on every run.
__global__ void __launch_bounds__(256) diag_final_kernel(const double* __restrict__ part, int nlat, int nmesh,
                                                         double* __restrict__ out) {
    __shared__ double red[5][256];
    const int t = threadIdx.x;
    for (int g = 0; g < 2; ++g) {
        const double* p = part + (g ? 5 * (size_t)nlat : 0);
        const int n = g ? nmesh : nlat;
        double s[5] = {0, 0, 0, 0, 0};
        for (int k = t; k < n; k += 256)
#pragma unroll
            for (int c = 0; c < 5; ++c) s[c] += p[5 * (size_t)k + c];
#pragma unroll
        for (int c = 0; c < 5; ++c) red[c][t] = s[c];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w)
#pragma unroll
                for (int c = 0; c < 5; ++c) red[c][t] += red[c][t + w];
            __syncthreads();
        }
        if (t < 5) out[5 * g + t] = red[t][0];
        __syncthreads();
    }
}

__device__ inline double weight_of(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// full populations n_i = w_i rho0 + d_i (dev = 0), or the stored deviations
// d_i alone (dev = 1), which FP64 holds exactly in every storage form
template <int P>
__global__ void pops_to_f64_kernel(const BoxDev* __restrict__ B, int parity, double* __restrict__ out, int dev) {
    typedef typename Prec<P>::S S;
    const int N = B->N;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)19 * N) return;
    const int i = (int)(k / N), p = (int)(k - (size_t)i * N);
    const S* src = (const S*)B->f[parity];
    const double d = (double)dec<P>(pop_load(src, i, p), B->st_inv);
    out[k] = dev ? d : weight_of(i) * B->rho0 + d;
}

template <int P>
__global__ void f64_to_pops_kernel(const BoxDev* __restrict__ B, int parity, const double* __restrict__ in,
                                   int dev) {
    typedef typename Prec<P>::S S;
    typedef typename Prec<P>::R R;
    const int N = B->N;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)19 * N) return;
    const int i = (int)(k / N), p = (int)(k - (size_t)i * N);
    S* dst = (S*)B->f[parity];
    pop_store(dst, i, p, enc<P>((R)(dev ? in[k] : in[k] - weight_of(i) * B->rho0), B->st_scale));
}

template <int P>
__global__ void moments_kernel(const BoxDev* __restrict__ B, int parity, double* __restrict__ rho,
                               double* __restrict__ u) {
    typedef typename Prec<P>::S S;
    const int N = B->N;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    if (B->btype && B->btype[p]) {  // obstacle node: rho0 and the wall velocity
        const double* uw = B->wall_u + 3 * B->btype[p];
        if (rho) rho[p] = B->rho0;
        if (u) {
            u[p] = uw[0];
            u[N + p] = uw[1];
            u[2 * N + p] = uw[2];
        }
        return;
    }
    const S* src = (const S*)B->f[parity];
    double d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = (double)dec<P>(pop_load(src, i, p), B->st_inv);
    double dr = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        dr += d[i];
        jx += cx(i) * d[i];
        jy += cy(i) * d[i];
        jz += cz(i) * d[i];
    }
    const double r = B->rho0 + dr;
    if (rho) rho[p] = r;
    if (u) {
        u[p] = (jx + 0.5 * B->g[0]) / r;
        u[N + p] = (jy + 0.5 * B->g[1]) / r;
        u[2 * N + p] = (jz + 0.5 * B->g[2]) / r;
    }
}

// plain streaming copy, 16 bytes per thread (bandwidth reference)
__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float4*)src,
                       (float4*)dst, n);
    return hipGetLastError();
}

#define OIF_DISPATCH_P(prec, KER, grid, blk, s, ...)                                               \
    switch (prec) {                                                                              \
        case PREC_FP64: hipLaunchKernelGGL(KER<PREC_FP64>, grid, blk, 0, s, __VA_ARGS__); break; \
        case PREC_FP32: hipLaunchKernelGGL(KER<PREC_FP32>, grid, blk, 0, s, __VA_ARGS__); break; \
        case PREC_FP16: hipLaunchKernelGGL(KER<PREC_FP16>, grid, blk, 0, s, __VA_ARGS__); break; \
        case PREC_BF16: hipLaunchKernelGGL(KER<PREC_BF16>, grid, blk, 0, s, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                                    \
    }

template <int P>
void launch_lb_p(const LbLaunch& L) {
#define OIF_LB(O, A, M, NT)                                                                                     \
    hipLaunchKernelGGL((lb_kernel<P, O, A, M, NT>), dim3(L.nblocks), dim3(L.block), 0, L.stream, L.boxes, L.work, \
                       L.nblocks, L.parity, L.remap, L.mode)
#define OIF_LB_M(O, A, NT)             \
    if (L.mrt) OIF_LB(O, A, true, NT); \
    else OIF_LB(O, A, false, NT)
    // the split step's two launches keep ordinary reads
    const bool all = L.mode == LB_ALL;
    if (L.obstacles) {
        if (!all) OIF_LB_M(true, false, false);
        else if (L.nt) OIF_LB_M(true, true, true);
        else OIF_LB_M(true, true, false);
    } else {
        if (!all) OIF_LB_M(false, false, false);
        else if (L.nt) OIF_LB_M(false, true, true);
        else OIF_LB_M(false, true, false);
    }
#undef OIF_LB_M
#undef OIF_LB
}

hipError_t launch_lb(const LbLaunch& L) {
    switch (L.precision) {
        case PREC_FP64: launch_lb_p<PREC_FP64>(L); break;
        case PREC_FP32: launch_lb_p<PREC_FP32>(L); break;
        case PREC_FP16: launch_lb_p<PREC_FP16>(L); break;
        case PREC_BF16: launch_lb_p<PREC_BF16>(L); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_diag_lattice(const BoxDev* box_dev, int precision, int parity, double* partials,
                               int nblocks, hipStream_t s) {
    // 1024 threads per block: sixteen waves per compute unit keep enough
    // population loads in flight over the grid-stride loop
    OIF_DISPATCH_P(precision, diag_lattice_kernel, dim3(nblocks), dim3(1024), s, box_dev, parity, partials);
    return hipGetLastError();
}

hipError_t launch_diag_final(const double* partials, int nlat, int nmesh, double* out, hipStream_t s) {
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, partials, nlat, nmesh, out);
    return hipGetLastError();
}

hipError_t launch_pops_to_f64(const BoxDev* box_dev, int N, int precision, int parity, double* out,
                              int deviations, hipStream_t s) {
    const size_t n = (size_t)19 * N;
    OIF_DISPATCH_P(precision, pops_to_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), s, box_dev,
                   parity, out, deviations);
    return hipGetLastError();
}

hipError_t launch_f64_to_pops(const BoxDev* box_dev, int N, int precision, int parity,
                              const double* in, int deviations, hipStream_t s) {
    const size_t n = (size_t)19 * N;
    OIF_DISPATCH_P(precision, f64_to_pops_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), s, box_dev,
                   parity, in, deviations);
    return hipGetLastError();
}

hipError_t launch_moments(const BoxDev* box_dev, int N, int precision, int parity, double* rho,
                          double* u, hipStream_t s) {
    OIF_DISPATCH_P(precision, moments_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), s, box_dev,
                   parity, rho, u);
    return hipGetLastError();
}

}  // namespace oif
