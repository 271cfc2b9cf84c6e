// mesh_kernels.hip -- membrane forces, fluid coupling and mesh integration
// (paper: Section "Elastic interactions" for the stretching, bending, local
// area, global area and volume forces; Section "Method" for the IB point
// dynamics, eq. newton, and the drag coupling, eq. dragforce, with linear
// interpolation of the fluid velocity and distribution of the reaction).
//
// One workgroup per object.  Its node positions are staged in LDS (FP64), then
//   1. per triangle: unit inward normal, area, (S - S0)/S; FP64 block sums of
//      the object's area and volume (divergence theorem, signed tetrahedra);
//   2. per edge: the stretching coefficient from the strain (L - L0)/L0 and
//      the bending magnitude from theta - theta0, both formed in FP64 so the
//      cancellation near the relaxed shape keeps its digits;
//   3. per node: gather of its edge, hinge and triangle contributions in a
//      fixed order (deterministic, no atomics), trilinear interpolation of the
//      fluid velocity from the 8 surrounding nodes, drag, symplectic Euler
//      update, and spreading of the reaction to the 8 nodes (int64 fixed-point
//      atomics: one word per component in the FP32 forms, a 2^-30 / 2^-80
//      pair of words in the FP64 form; exact, so order-independent) with the
//      nodes' mask bits set.
// With velocity Verlet (the integrator of the paper's engine) the staged
// positions are first advanced by the half-step velocity V + F_last/(2m), the
// forces and the drag are taken there (drag at the half-step velocity), and
// the update is the second half kick; the total force is kept for the next
// step.
// Meshes whose arrays do not fit in LDS use a per-object global scratch area
// with the same layout; when their patches fit in LDS, they are split over
// several workgroups per object (the area and volume summed over slices of
// the triangles, then each compact patch of nodes run as an LDS-resident
// object on its own sub-template, the slices' sums added in a fixed order).
#include <vector>

#include "mesh_device.h"

namespace oif {
namespace {

using namespace dev;

// the per-object routine and its helpers: mesh_device.h

// Below FP64, registers are capped for six waves per SIMD: two objects of up
// to 768 threads then share a compute unit (both meshes fit its LDS), so each
// phase's loops over triangles, edges and nodes take fewer rounds.
template <int P, bool USE_LDS, bool CONS, bool CPL, bool LISTS>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(P == PREC_FP64 ? 1 : 6)))
mesh_kernel(const ObjDev<typename Prec<P>::R>* __restrict__ objs, int parity, int mark_next) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int bid = blockIdx.x;
    mesh_object<P, USE_LDS, CONS, CPL, PH_ALL, LISTS>(objs[bid], smem, parity, mark_next);
}

// Meshes too large for LDS whose patches fit there, split over several
// workgroups per object: the sums launch (PH_SUMS) and then the patch launch
// (PH_PATCH), one workgroup per (object, slice) in `work`.
template <int P, bool CONS, int PH, bool LISTS>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(P == PREC_FP64 ? 1 : 6)))
mesh_split_kernel(const ObjDev<typename Prec<P>::R>* __restrict__ objs, const int2* __restrict__ work, int parity,
                  int mark_next) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 w = work[blockIdx.x];
    mesh_object<P, PH == PH_PATCH, CONS, PH != PH_PATCH, PH, LISTS>(objs[w.x], smem, parity, mark_next, w.y);
}

// Touch bits of a step of parity `parity` from the current positions (split
// stepping, when the membrane kernel of the previous step did not mark them).
// One workgroup per object.
template <typename R>
__global__ void __launch_bounds__(256) mark_kernel(const ObjDev<R>* __restrict__ objs, int parity, int cap) {
    extern __shared__ unsigned bits[];  // cap bits
    __shared__ int bbox[6];
    const ObjDev<R>& O = objs[blockIdx.x];
    const gptr<const BoxDev> B = (gptr<const BoxDev>)O.box;
    mark_object(O.X, nullptr, O.t->nv, O.anchor, B, min(O.t->ucap, cap), bits, bbox, B->touch[parity]);
}

template <typename R>
__global__ void __launch_bounds__(256)
diag_mesh_kernel(const ObjDev<R>* __restrict__ objs, double* __restrict__ part) {
    __shared__ double red[16];
    const ObjDev<R>& O = objs[blockIdx.x];
    const int nv = O.t->nv;
    double vx = 0, vy = 0, vz = 0, bad = 0;
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        const double a = O.V[3 * v], b = O.V[3 * v + 1], c = O.V[3 * v + 2];
        vx += a; vy += b; vz += c;
        if (!isfinite(a + b + c) || !isfinite(O.X[3 * v] + O.X[3 * v + 1] + O.X[3 * v + 2])) bad = 1.0;
    }
    const double m = O.mass;
    const double s0 = block_sum(vx, red), s1 = block_sum(vy, red), s2 = block_sum(vz, red),
                 s3 = block_sum(bad, red);
    if (threadIdx.x == 0) {
        double* o = part + 5 * blockIdx.x;
        o[0] = 0.0; o[1] = m * s0; o[2] = m * s1; o[3] = m * s2; o[4] = s3;
    }
}

template <int P, bool LISTS>
hipError_t launch_mesh_pl(const MeshLaunch& L) {
    typedef typename Prec<P>::R R;
    const ObjDev<R>* objs = (const ObjDev<R>*)L.objs;
    const dim3 g(L.nobj), b(L.block);
    if (L.work) {
        const dim3 gw(L.nwork);
        if (L.conservative) {
            hipLaunchKernelGGL((mesh_split_kernel<P, true, PH_SUMS, LISTS>), gw, b, L.split_lds, L.stream, objs,
                               L.work, L.parity, L.mark_next);
            hipLaunchKernelGGL((mesh_split_kernel<P, true, PH_PATCH, LISTS>), gw, b, L.split_lds, L.stream, objs,
                               L.work, L.parity, L.mark_next);
        } else {
            hipLaunchKernelGGL((mesh_split_kernel<P, false, PH_SUMS, LISTS>), gw, b, L.split_lds, L.stream, objs,
                               L.work, L.parity, L.mark_next);
            hipLaunchKernelGGL((mesh_split_kernel<P, false, PH_PATCH, LISTS>), gw, b, L.split_lds, L.stream, objs,
                               L.work, L.parity, L.mark_next);
        }
    } else if (L.lds_bytes > 0) {
        if (L.conservative)
            hipLaunchKernelGGL((mesh_kernel<P, true, true, false, LISTS>), g, b, L.lds_bytes, L.stream, objs, L.parity,
                               L.mark_next);
        else
            hipLaunchKernelGGL((mesh_kernel<P, true, false, false, LISTS>), g, b, L.lds_bytes, L.stream, objs, L.parity,
                               L.mark_next);
    } else if (L.cpl_lds_bytes > 0) {
        if (L.conservative)
            hipLaunchKernelGGL((mesh_kernel<P, false, true, true, LISTS>), g, b, L.cpl_lds_bytes, L.stream, objs,
                               L.parity, L.mark_next);
        else
            hipLaunchKernelGGL((mesh_kernel<P, false, false, true, LISTS>), g, b, L.cpl_lds_bytes, L.stream, objs,
                               L.parity, L.mark_next);
    } else {
        if (L.conservative)
            hipLaunchKernelGGL((mesh_kernel<P, false, true, false, LISTS>), g, b, 0, L.stream, objs, L.parity,
                               L.mark_next);
        else
            hipLaunchKernelGGL((mesh_kernel<P, false, false, false, LISTS>), g, b, 0, L.stream, objs, L.parity,
                               L.mark_next);
    }
    return hipGetLastError();
}

template <int P>
hipError_t launch_mesh_p(const MeshLaunch& L) {
    return L.lists ? launch_mesh_pl<P, true>(L) : launch_mesh_pl<P, false>(L);
}

// every membrane kernel variant that may take more than the default dynamic
// LDS, for one precision
template <int P, bool LISTS>
void dynlds_kernels(std::vector<const void*>& v) {
    v.push_back((const void*)mesh_kernel<P, true, false, false, LISTS>);
    v.push_back((const void*)mesh_kernel<P, true, true, false, LISTS>);
    v.push_back((const void*)mesh_kernel<P, false, false, true, LISTS>);
    v.push_back((const void*)mesh_kernel<P, false, true, true, LISTS>);
    v.push_back((const void*)mesh_split_kernel<P, false, PH_SUMS, LISTS>);
    v.push_back((const void*)mesh_split_kernel<P, true, PH_SUMS, LISTS>);
    v.push_back((const void*)mesh_split_kernel<P, false, PH_PATCH, LISTS>);
    v.push_back((const void*)mesh_split_kernel<P, true, PH_PATCH, LISTS>);
}

}  // namespace

size_t mesh_lds_bytes(int precision, int nv, int nt, int ne, int ucap, int ccap, int cons) {
    return mesh_layout(precision == PREC_FP64 ? sizeof(double) : sizeof(float), nv, nt, ne, ucap, ccap, cons)
        .total;
}

size_t mesh_cpl_lds_bytes(int precision, int nv, int nt, int ne, int ucap, int ccap, int cons) {
    const MeshLayout L =
        mesh_layout(precision == PREC_FP64 ? sizeof(double) : sizeof(float), nv, nt, ne, ucap, ccap, cons);
    return align16(L.gacc + (size_t)ccap * (precision == PREC_FP64 ? 6 : 3) * 8) - L.need;
}

hipError_t launch_mesh(const MeshLaunch& L) {
    if (L.work ? L.nwork <= 0 : L.nobj <= 0) return hipSuccess;
    switch (L.precision) {
        case PREC_FP64: return launch_mesh_p<PREC_FP64>(L);
        case PREC_FP32: return launch_mesh_p<PREC_FP32>(L);
        case PREC_FP16: return launch_mesh_p<PREC_FP16>(L);
        case PREC_BF16: return launch_mesh_p<PREC_BF16>(L);
        default: return hipErrorInvalidValue;
    }
}

// Let the LDS-resident variants use up to `bytes` of dynamic LDS per workgroup.
hipError_t mesh_set_max_lds(size_t bytes) {
    hipError_t e = hipSuccess;
    std::vector<const void*> fns;
    dynlds_kernels<PREC_FP64, false>(fns);
    dynlds_kernels<PREC_FP32, false>(fns);
    dynlds_kernels<PREC_FP16, false>(fns);
    dynlds_kernels<PREC_BF16, false>(fns);
    dynlds_kernels<PREC_FP64, true>(fns);
    dynlds_kernels<PREC_FP32, true>(fns);
    dynlds_kernels<PREC_FP16, true>(fns);
    dynlds_kernels<PREC_BF16, true>(fns);
    for (const void* f : fns) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (r != hipSuccess) e = r;
    }
    return e;
}

hipError_t launch_mark(const void* objs, int nobj, int precision, size_t lds_bytes, int parity,
                       hipStream_t s) {
    if (nobj <= 0) return hipSuccess;
    const int cap = (int)(lds_bytes / 4) * 32;
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(mark_kernel<double>, dim3(nobj), dim3(256), lds_bytes, s, (const ObjDev<double>*)objs,
                           parity, cap);
    else
        hipLaunchKernelGGL(mark_kernel<float>, dim3(nobj), dim3(256), lds_bytes, s, (const ObjDev<float>*)objs,
                           parity, cap);
    return hipGetLastError();
}

hipError_t launch_diag_mesh(const void* objs, int nobj, int precision, double* partials, hipStream_t s) {
    if (nobj <= 0) return hipSuccess;
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(diag_mesh_kernel<double>, dim3(nobj), dim3(256), 0, s, (const ObjDev<double>*)objs,
                           partials);
    else
        hipLaunchKernelGGL(diag_mesh_kernel<float>, dim3(nobj), dim3(256), 0, s, (const ObjDev<float>*)objs,
                           partials);
    return hipGetLastError();
}

}  // namespace oif
