// mesh_device.h -- device routines of the membrane forces, fluid coupling
// and mesh integration (paper: Section "Elastic interactions" for the
// stretching, bending, local area, global area and volume forces; Section
// "Method" for the IB point dynamics, eq. newton, and the drag coupling,
// eq. dragforce, with linear interpolation of the fluid velocity and
// distribution of the reaction), shared by the membrane kernel and the
// persistent batch kernel.  The outline of the per-object routine is in
// mesh_kernels.hip.
#pragma once

#include <limits.h>

#include "device_common.h"
#include "fixed_point.h"

namespace oif {
namespace dev {

// Accumulation of the reaction force handed to the fluid.  FP32 forms: int64
// fixed point with resolution 2^-e, so sums are exact and independent of the
// order in which mesh nodes add (bitwise reproducible); FP64 form: FP64.
template <int P>
struct Acc {
    // FP32 forms: one int64 word per component, the value times 2^fixed_point_exp
    typedef unsigned long long T;
    static constexpr int WC = 1;    // words per component
    static constexpr int SLOT = 4;  // words per node of G (x, y, z, unused)
    __device__ static void convert(float v, double scale, T* out, unsigned& fl) {
        const double a = (double)v * scale;
        // below 2^55 units, so a sum of up to 256 values stays in the int64 range
        if (!(fabs(a) < 0x1p55)) {  // out of range or not finite
            fl |= ST_OVERFLOW;
            out[0] = 0ull;
            return;
        }
        out[0] = (T)__double2ll_rn(a);
    }
};

template <>
struct Acc<PREC_FP64> {
    // FP64 form: two int64 words per component, the value split into a
    // multiple of 2^-30 and the remainder in units of 2^-80.  Both integer
    // sums are exact, so the spread force does not depend on the order of the
    // additions (as in the FP32 forms); a value is rounded only below 2^-80,
    // and |value| < 2^25 (else the overflow flag), which leaves room for
    // sums of 256 values.
    typedef unsigned long long T;
    static constexpr int WC = 2;
    static constexpr int SLOT = 8;  // x hi, x lo, y hi, y lo, z hi, z lo, two unused
    __device__ static void convert(double v, double, T* out, unsigned& fl) {
        long long hi, lo;
        if (!fx_split(v, hi, lo)) fl |= ST_OVERFLOW;
        out[0] = (T)hi;
        out[1] = (T)lo;
    }
};

// Add a reaction force to a node's LDS accumulator (3 * WC words).
template <int P>
__device__ __forceinline__ unsigned acc_add(typename Acc<P>::T* acc, typename Prec<P>::R x, typename Prec<P>::R y,
                                            typename Prec<P>::R z, double scale) {
    constexpr int WC = Acc<P>::WC;
    unsigned fl = 0;
    typename Acc<P>::T v[3 * WC];
    Acc<P>::convert(x, scale, v, fl);
    Acc<P>::convert(y, scale, v + WC, fl);
    Acc<P>::convert(z, scale, v + 2 * WC, fl);
#pragma unroll
    for (int w = 0; w < 3 * WC; ++w) atomicAdd(acc + w, v[w]);
    return fl;
}

// Add a node's summed reaction (3 * WC words) to G at lattice node q and set
// its mask bit.
template <int P>
__device__ __forceinline__ void acc_flush(gptr<const BoxDev> B, int parity, int q, const typename Acc<P>::T* v) {
    constexpr int WC = Acc<P>::WC;
    typedef typename Acc<P>::T T;
    T any = 0ull;
#pragma unroll
    for (int w = 0; w < 3 * WC; ++w) any |= v[w];
    if (any == 0ull) return;
    T* G = (T*)B->G[parity] + Acc<P>::SLOT * (size_t)q;
#pragma unroll
    for (int w = 0; w < 3 * WC; ++w)
        if (v[w]) gatomic_add(G + w, v[w]);
    gatomic_or(B->mask + (q >> 6), 1ull << (q & 63));
}

// Lattice index of the (unwrapped) node (gx, gy, gz): periodic in x and y,
// periodic or clamped to the walls in z.
__device__ __forceinline__ int lattice_node(gptr<const BoxDev> B, int gx, int gy, int gz) {
    const int nxb = B->nx, nyb = B->ny, nzb = B->nz;
    gx %= nxb;
    gx += gx < 0 ? nxb : 0;
    gy %= nyb;
    gy += gy < 0 ? nyb : 0;
    if (B->walls_z) {
        gz = gz < 0 ? 0 : (gz >= nzb ? nzb - 1 : gz);
    } else {
        gz %= nzb;
        gz += gz < 0 ? nzb : 0;
    }
    return (gz * nyb + gy) * nxb + gx;
}

// q = a / d, r = a % d for 0 <= a < 2^20 and 0 < d, without an integer
// division: the float estimate a * (1/d) is within one of the quotient.
__device__ __forceinline__ void divmod_small(int a, int d, float rd, int& q, int& r) {
    q = (int)((float)a * rd);
    r = a - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
}

// a mod n in [0, n)
__device__ __forceinline__ int wrap_mod(int a, int n) {
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// Lower corner of the 2x2x2 stencil of a mesh node at (px, py, pz): nodes sit
// at cell centres, so the stencil starts at floor(x - 1/2) per axis (plus the
// object's integer anchor).  False for a non-finite or runaway position,
// which gets no stencil.
__device__ __forceinline__ bool stencil_corner(double px, double py, double pz, const int* anchor, int (&b)[3]) {
    const double sx = px - 0.5, sy = py - 0.5, sz = pz - 0.5;
    if (!(fabs(sx) < 1e7 && fabs(sy) < 1e7 && fabs(sz) < 1e7)) return false;
    b[0] = anchor[0] + (int)floor(sx);
    b[1] = anchor[1] + (int)floor(sy);
    b[2] = anchor[2] + (int)floor(sz);
    return true;
}

// Stencil marking of one object for split stepping: every lattice node inside
// the 2x2x2 stencil of a finite node position gets its bit in `touch`.  The
// object's stencil box is marked in the bitmask `bits` ((ucap + 31)/32 words)
// first when it fits, so each touched node costs one global atomic however
// many stencils contain it; otherwise every corner goes to `touch` directly.
// Called by the whole workgroup.  The nodes marked: 0 .. nv - 1, or
// order[0 .. nv - 1] when order is not null.
__device__ void mark_object(const double* pos, const int* order, int nv, const int* anchor, gptr<const BoxDev> B,
                            int ucap, unsigned* bits, int* bbox, unsigned long long* touch) {
    __syncthreads();  // earlier users of bits and bbox are done
    if (threadIdx.x == 0) {
        bbox[0] = bbox[1] = bbox[2] = INT_MAX;
        bbox[3] = bbox[4] = bbox[5] = INT_MIN;
    }
    __syncthreads();
    int blo[3] = {INT_MAX, INT_MAX, INT_MAX}, bhi[3] = {INT_MIN, INT_MIN, INT_MIN};
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const int v = order ? gld(order + i) : i;
        const double sx = pos[3 * v] - 0.5, sy = pos[3 * v + 1] - 0.5, sz = pos[3 * v + 2] - 0.5;
        if (!(fabs(sx) < 1e7 && fabs(sy) < 1e7 && fabs(sz) < 1e7)) continue;
        const int bx = anchor[0] + (int)floor(sx), by = anchor[1] + (int)floor(sy),
                  bz = anchor[2] + (int)floor(sz);
        blo[0] = min(blo[0], bx); blo[1] = min(blo[1], by); blo[2] = min(blo[2], bz);
        bhi[0] = max(bhi[0], bx); bhi[1] = max(bhi[1], by); bhi[2] = max(bhi[2], bz);
    }
    wave_bbox_to_block(blo, bhi, bbox);
    __syncthreads();
    const int ox = bbox[0], oy = bbox[1], oz = bbox[2];
    if (bbox[3] < bbox[0]) return;  // no finite node (block-uniform)
    const long long exl = (long long)bbox[3] - ox + 2, eyl = (long long)bbox[4] - oy + 2,
                    ezl = (long long)bbox[5] - oz + 2;
    if (exl * eyl * ezl <= (long long)ucap) {
        const int ex = (int)exl, exy = (int)(exl * eyl), vol = (int)(exl * eyl * ezl);
        for (int k = threadIdx.x; k < (vol + 31) / 32; k += blockDim.x) bits[k] = 0u;
        __syncthreads();
        for (int i = threadIdx.x; i < nv; i += blockDim.x) {
            const int v = order ? gld(order + i) : i;
            const double sx = pos[3 * v] - 0.5, sy = pos[3 * v + 1] - 0.5, sz = pos[3 * v + 2] - 0.5;
            if (!(fabs(sx) < 1e7 && fabs(sy) < 1e7 && fabs(sz) < 1e7)) continue;
            const int b0 = (anchor[2] + (int)floor(sz) - oz) * exy + (anchor[1] + (int)floor(sy) - oy) * ex +
                           (anchor[0] + (int)floor(sx) - ox);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = (kk + (int)threadIdx.x) & 7;
                const int idx = b0 + (k >> 2) * exy + ((k >> 1) & 1) * ex + (k & 1);
                atomicOr(&bits[idx >> 5], 1u << (idx & 31));
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < vol; idx += blockDim.x) {
            if (!((bits[idx >> 5] >> (idx & 31)) & 1u)) continue;
            const int q = lattice_node(B, ox + idx % ex, oy + (idx / ex) % (int)eyl, oz + idx / exy);
            gatomic_or(touch + (q >> 6), 1ull << (q & 63));
        }
    } else {
        for (int i = threadIdx.x; i < nv; i += blockDim.x) {
            const int v = order ? gld(order + i) : i;
            const double sx = pos[3 * v] - 0.5, sy = pos[3 * v + 1] - 0.5, sz = pos[3 * v + 2] - 0.5;
            if (!(fabs(sx) < 1e7 && fabs(sy) < 1e7 && fabs(sz) < 1e7)) continue;
            const int bx = anchor[0] + (int)floor(sx), by = anchor[1] + (int)floor(sy),
                      bz = anchor[2] + (int)floor(sz);
            for (int k = 0; k < 8; ++k) {
                const int q = lattice_node(B, bx + (k & 1), by + ((k >> 1) & 1), bz + (k >> 2));
                gatomic_or(touch + (q >> 6), 1ull << (q & 63));
            }
        }
    }
}

// CONS: some object of the launch may use the conservative force model (each
// object's template says whether it does); without it that code is left out.
// CPL (meshes too large for LDS only): the coupling area alone sits in LDS, so
// that the stencil-bit ORs and the per-node force sums, whose addresses many
// mesh nodes share, are LDS and not global atomics.
// PH: the whole object in one workgroup (PH_ALL), or one of the two launches
// that split it over T->nslice workgroups (meshes too large for LDS whose
// patches fit there): PH_SUMS, the area and volume sums of slice `slice` of
// the triangles, left in the object's scratch; PH_PATCH, the forces, coupling
// and update of patch `slice` of the nodes, run as an LDS-resident object on
// the patch's sub-template (T->subs[slice]: the patch's nodes first, then the
// other nodes its triangles and hinges reach, with the triangles and hinges
// its nodes' gathers read and incidence lists in local numbering), after the
// area and volume are summed from the slices in a fixed order.
// LISTS: some box of the launch has the membrane kernel clear its coupling
// force (BoxDev::g_by_mesh); without it the list code is left out.
// The membrane forces, coupling and update of object O by the whole
// workgroup; smem is the workgroup's dynamic LDS.
template <int P, bool USE_LDS, bool CONS, bool CPL, int PH = PH_ALL, bool LISTS = true>
__device__ __forceinline__ void mesh_object(const ObjDev<typename Prec<P>::R>& O, unsigned char* smem, int parity,
                                            int mark_next, int slice = 0) {
    constexpr bool SPLIT = PH != PH_ALL;
    static_assert(PH != PH_SUMS || (!USE_LDS && CPL), "sums launch: positions alone in LDS");
    static_assert(PH != PH_PATCH || (USE_LDS && !CPL), "patch launch: the patch's sub-template in LDS");
    typedef typename Prec<P>::S S;
    typedef typename Prec<P>::R R;
    __shared__ double red[16];

    const gptr<const TmplDev<R>> Tp = (gptr<const TmplDev<R>>)O.t;  // the object's template
    const gptr<const TmplDev<R>> T = PH == PH_PATCH ? (gptr<const TmplDev<R>>)(Tp->subs + slice) : Tp;
    const gptr<const BoxDev> B = (gptr<const BoxDev>)O.box;
    const int nv = T->nv, nt = T->nt, ne = T->ne;
    const int ucap = T->ucap, ccap = T->ccap;
    const int cons = CONS ? T->conservative : 0;
    const MeshLayout lay = mesh_layout(sizeof(R), nv, nt, ne, ucap, ccap, cons);
    unsigned char* base = USE_LDS ? smem : O.scratch;
    R* fs = (R*)(base + lay.fs);      // [nodes of the launch][3]: elastic force
    // [nv][3]: positions (forces phase); the sums launch keeps them alone in LDS
    double* xs = PH == PH_SUMS ? (double*)smem : (double*)(base + lay.xs);
    R* tn = (R*)(base + lay.tn);      // [nt][4]: unit inward normal, area
    R* tr = (R*)(base + lay.tr);      // [nt]: (S - S0)/S
    R* se = (R*)(base + lay.se);      // [ne]: ks kappa strain / L
    R* fh = (R*)(base + lay.fh);      // [ne]: kb (theta - theta0)/theta0
    // coupling area: over the positions and the forces-phase arrays, or alone
    // in LDS (CPL)
    auto carea = [&](size_t off) -> unsigned char* {
        return (!USE_LDS && CPL) ? smem + (off - lay.need) : base + off;
    };
    // the nodes this launch updates: all, or the patch (its sub-template's
    // first nodes; T->order maps them to the object's node numbers)
    const int nsl = SPLIT ? T->nslice : 1;
    const int n0 = 0;
    const int nn = PH == PH_PATCH ? gld(T->slice_off + 1) : nv;
    auto node_of = [&](int i) -> int { return PH == PH_PATCH ? gld(T->order + i) : i; };
    // the slices' area and volume sums, after the object's mesh layout in its scratch
    double* part = SPLIT ? (double*)(O.scratch + split_part_offset(mesh_layout(sizeof(R), Tp->nv, Tp->nt, Tp->ne,
                                                                                ucap, ccap, cons)))
                         : nullptr;  // [nslice][2]

    // When the membrane kernel clears G (B->g_by_mesh): the G slots this object
    // added to in the previous step (G[parity ^ 1], which the lattice kernel
    // has read by now) are zeroed for the step after this one, from the lists
    // the previous step kept (per slice; a whole-object workgroup takes all of
    // them, since the previous step may have run split), and the previous
    // step's flag is reset.  This step's lists start empty.  (Otherwise the
    // lattice kernel clears G and no lists are kept.)
    const bool lists = LISTS && B->g_by_mesh != 0;
    const int kq = T->nslice;
    const size_t qstride = (size_t)ccap + 1;
    if (PH != PH_SUMS && lists) {
        const int np = parity ^ 1;
        unsigned char* Gp = (unsigned char*)B->G[np];
        for (int sl = SPLIT ? slice : 0; sl < (SPLIT ? slice + 1 : kq); ++sl) {
            const int* qo = O.qsave + ((size_t)np * kq + sl) * qstride;
            const int cnt = min(gld(qo), ccap);
            for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
                unsigned long long* g = (unsigned long long*)Gp + Acc<P>::SLOT * (size_t)gld(qo + 1 + k);
#pragma unroll
                for (int w = 0; w < 3 * Acc<P>::WC; ++w) gst(g + w, 0ull);
            }
        }
        if (threadIdx.x == 0) gst(B->gclear + np, 0u);
        if ((int)threadIdx.x < (SPLIT ? 1 : kq))
            gst(O.qsave + ((size_t)parity * kq + (SPLIT ? slice : (int)threadIdx.x)) * qstride, 0);
    }
    unsigned* need = (unsigned*)carea(lay.need);  // coupling phase: stencil-box bits
    __shared__ int bbox[6];
    __shared__ int ncomp;

    // Position of node k (component-wise index) the forces and the drag are
    // taken at: X, or with velocity Verlet X + (V + F_last/(2m)), the
    // half-step velocity rounded once.  Staged in LDS for the forces phase and
    // formed again from HBM by the coupling phase (the same expression, so the
    // same bits).
    const R half_im = R(0.5) * O.inv_mass;
    auto stage = [&](int k) -> double {
        return O.F ? gld(O.X + k) + (double)fmadd(gld(O.F + k), half_im, gld(O.V + k)) : gld(O.X + k);
    };
    for (int k = threadIdx.x; k < 3 * nv; k += blockDim.x)
        xs[k] = PH == PH_PATCH ? stage(3 * gld(T->order + k / 3) + k % 3) : stage(k);
    if (threadIdx.x == 0) {
        bbox[0] = bbox[1] = bbox[2] = INT_MAX;
        bbox[3] = bbox[4] = bbox[5] = INT_MIN;
    }
    __syncthreads();

    // 1. triangles
    // (S - S0 is formed as (S^2 - S0^2)/(S + S0): the cancelling difference in
    // FP64 multiply-adds, the square root and division in the arithmetic type)
    double sdarea = 0.0, svol = 0.0;
    {
        // node 0 of the object: the apex of the signed tetrahedra, and the
        // origin the triangles' edge vectors are taken from in every launch
        const double r0x = PH == PH_PATCH ? stage(0) : xs[0], r0y = PH == PH_PATCH ? stage(1) : xs[1],
                     r0z = PH == PH_PATCH ? stage(2) : xs[2];
        const int t0 = PH == PH_SUMS ? (int)((long long)nt * slice / nsl) : 0;
        const int t1 = PH == PH_SUMS ? (int)((long long)nt * (slice + 1) / nsl) : nt;
        for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
            const int a = gld(T->tri + 3 * t), b = gld(T->tri + 3 * t + 1), c = gld(T->tri + 3 * t + 2);
            const double ax = xs[3 * a] - r0x, ay = xs[3 * a + 1] - r0y, az = xs[3 * a + 2] - r0z;
            const double bx = xs[3 * b] - r0x, by = xs[3 * b + 1] - r0y, bz = xs[3 * b + 2] - r0z;
            const double qx = xs[3 * c] - r0x, qy = xs[3 * c + 1] - r0y, qz = xs[3 * c + 2] - r0z;
            const double abx = bx - ax, aby = by - ay, abz = bz - az;
            const double acx = qx - ax, acy = qy - ay, acz = qz - az;
            const double nx_ = aby * acz - abz * acy;
            const double ny_ = abz * acx - abx * acz;
            const double nz_ = abx * acy - aby * acx;
            const double n2 = nx_ * nx_ + ny_ * ny_ + nz_ * nz_;  // 4 S^2
            const R len = sqrt((R)n2);
            const R S = R(0.5) * len;
            const double S0 = gld(T->S0 + t);
            const R dS = (R)(0.25 * n2 - S0 * S0) / (S + (R)S0);
            if (PH != PH_SUMS) {  // the sums launch keeps the sums only
                tn[4 * t + 0] = (R)nx_ / len;
                tn[4 * t + 1] = (R)ny_ / len;
                tn[4 * t + 2] = (R)nz_ / len;
                tn[4 * t + 3] = S;
                tr[t] = dS / S;
            }
            sdarea += (double)dS;
            // signed tetrahedron (node 0, a, b, c): inward orientation gives -6 V
            const double cxx = by * qz - bz * qy, cyy = bz * qx - bx * qz, czz = bx * qy - by * qx;
            svol -= (ax * cxx + ay * cyy + az * czz) / 6.0;
        }
    }
    double dSg, Vol;  // Sg - Sg0, volume
    if (PH == PH_ALL) {
        dSg = block_sum(sdarea, red);
        Vol = block_sum(svol, red);
    } else if (PH == PH_SUMS) {
        dSg = block_sum(sdarea, red);
        Vol = block_sum(svol, red);
        if (threadIdx.x == 0) {
            gst(part + 2 * slice, dSg);
            gst(part + 2 * slice + 1, Vol);
        }
        return;  // the patch launch reads the slices' sums
    } else {
        // the slices' sums, added in slice order (the same bits in every
        // workgroup of the object)
        dSg = 0.0;
        Vol = 0.0;
        for (int k = 0; k < nsl; ++k) {
            dSg += gld(part + 2 * k);
            Vol += gld(part + 2 * k + 1);
        }
    }
    const double Sg = T->Sg0 + dSg;
    if (threadIdx.x == 0 && slice == 0 && O.geo) {
        gst(O.geo, Sg);
        gst(O.geo + 1, Vol);
    }

    // 2. edges: stretching coefficient and bending magnitude of each hinge
    const bool do_s = T->ks != 0.0, do_b = T->kb != 0.0;
    if (do_s || do_b) {
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            const int4 h = gld(T->hinge + e);  // (A, B, C, D): the edge is B -> C
            const double dx = xs[3 * h.z] - xs[3 * h.y], dy = xs[3 * h.z + 1] - xs[3 * h.y + 1],
                         dz = xs[3 * h.z + 2] - xs[3 * h.y + 2];
            const double L2 = dx * dx + dy * dy + dz * dz;
            const double L = sqrt(L2);
            if (do_s) {
                // strain (L - L0)/L0 = (L^2 - L0^2) / (L0 (L + L0))
                const double L0 = gld(T->L0 + e);
                const R strain = (R)(L2 - L0 * L0) / ((R)L0 * (R)(L + L0));
                R kap = R(1);
                if (!T->linear) {
                    const R lam = R(1) + strain, sl = sqrt(lam), l2 = lam * lam;
                    kap = (sl + R(1) / (l2 * sl)) / (lam + R(1) / (l2 * lam));
                }
                se[e] = (R)T->ks * kap * strain / (R)L;
            }
            if (do_b) {
                // normals of T1 = (A, B, C) and T2 = (D, C, B) (inward, unnormalised)
                const double* pa = &xs[3 * h.x];
                const double* pb = &xs[3 * h.y];
                const double* pc = &xs[3 * h.z];
                const double* pd = &xs[3 * h.w];
                const double u1x = pb[0] - pa[0], u1y = pb[1] - pa[1], u1z = pb[2] - pa[2];
                const double v1x = pc[0] - pa[0], v1y = pc[1] - pa[1], v1z = pc[2] - pa[2];
                const double n1x = u1y * v1z - u1z * v1y, n1y = u1z * v1x - u1x * v1z, n1z = u1x * v1y - u1y * v1x;
                const double u2x = pc[0] - pd[0], u2y = pc[1] - pd[1], u2z = pc[2] - pd[2];
                const double v2x = pb[0] - pd[0], v2y = pb[1] - pd[1], v2z = pb[2] - pd[2];
                const double n2x = u2y * v2z - u2z * v2y, n2y = u2z * v2x - u2x * v2z, n2z = u2x * v2y - u2y * v2x;
                const double mx = n1y * n2z - n1z * n2y, my = n1z * n2x - n1x * n2z, mz = n1x * n2y - n1y * n2x;
                // theta - pi = atan2((m . e), n1 . n2) for the unit vectors; the
                // difference to theta0 - pi is the angle of the relative rotation,
                // atan2(sin d, cos d), every term scaled by |N1| |N2| L > 0
                const double md = mx * dx + my * dy + mz * dz;
                const double dot = n1x * n2x + n1y * n2y + n1z * n2z;
                const double2 cs = gld(T->cs0 + e);  // cos, sin of theta0 - pi
                const R dth = atan2((R)(md * cs.x - dot * L * cs.y), (R)(dot * L * cs.x + md * cs.y));
                const R f = (R)T->kb * dth / (R)gld(T->theta0 + e);
                if (!cons) {
                    fh[e] = f;
                } else {
                    // gradient form: the wing factors c / h (c = hbar f, h = |N| / L
                    // the wing's distance from the edge line) and the positions a of
                    // the wings' feet on the edge, B + a (C - B)
                    const R c = (R)gld(T->hbar + e) * f;
                    const R nA = (R)sqrt(n1x * n1x + n1y * n1y + n1z * n1z);
                    const R nD = (R)sqrt(n2x * n2x + n2y * n2y + n2z * n2z);
                    const double abx = pa[0] - pb[0], aby = pa[1] - pb[1], abz = pa[2] - pb[2];
                    const double dbx = pd[0] - pb[0], dby = pd[1] - pb[1], dbz = pd[2] - pb[2];
                    R* q = fh + 4 * e;
                    q[0] = c * (R)L / nA;
                    q[1] = c * (R)L / nD;
                    q[2] = (R)((abx * dx + aby * dy + abz * dz) / L2);
                    q[3] = (R)((dbx * dx + dby * dy + dbz * dz) / L2);
                }
            }
        }
    }
    __syncthreads();

    const R cg = (R)(-T->kag * dSg / Sg);             // global area coefficient
    const R cv = (R)(-T->kv * (Vol - T->V0) / T->V0); // volume coefficient
    const R kal = (R)T->kal;
    const R third = R(1) / R(3);
    const int nxb = B->nx, nyb = B->ny, nzb = B->nz;
    const S* __restrict__ pop = (const S*)B->f[parity];
    const float inv = B->st_inv;
    const R gx_ = (R)B->g[0], gy_ = (R)B->g[1], gz_ = (R)B->g[2];
    const R rho0 = (R)B->rho0, xi = (R)B->xi;
    const unsigned char* bt = B->btype;  // obstacles (null: none)
    unsigned flags = 0;
    int blo[3] = {INT_MAX, INT_MAX, INT_MAX}, bhi[3] = {INT_MIN, INT_MIN, INT_MIN};

    // 3. nodes (in the patch launch the patch's nodes are the sub-template's
    // first nn nodes, so xs, the incidence lists and fs take the same index)
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
        const int v = i;
        const double px = xs[3 * v], py = xs[3 * v + 1], pz = xs[3 * v + 2];
        R Fx = 0, Fy = 0, Fz = 0;
        const int4 o0 = gld(T->n_off + v), o1 = gld(T->n_off + v + 1);
        if (do_s) {
            // F_v += ks kappa (L - L0)/L0 (x_u - x_v)/L  ("Stretching force")
#pragma unroll 2
            for (int k = o0.x; k < o1.x; ++k) {
                const int2 ie = gld(T->e_inc + k);
                const R s = se[ie.y];
                Fx += s * (R)(xs[3 * ie.x] - px);
                Fy += s * (R)(xs[3 * ie.x + 1] - py);
                Fz += s * (R)(xs[3 * ie.x + 2] - pz);
            }
        }
        if (do_b) {
            // wings along their triangle's normal, edge ends minus half the sum
            // ("Bending force"; conservative model: minus the wing forces split
            // by the positions of the wings' feet); the role picks the two
            // coefficients of the normals n1, n2
#pragma unroll 4
            for (int k = o0.y; k < o1.y; ++k) {
                const int4 r = gld(T->h_inc + k);
                const int role = r.x & 3;
                R a1, a2;
                if (!cons) {
                    const R f = fh[r.x >> 2];
                    const R hf = R(-0.5) * f;
                    a1 = role == 0 ? f : (role == 3 ? R(0) : hf);
                    a2 = role == 3 ? f : (role == 0 ? R(0) : hf);
                } else {
                    const R* q = fh + 4 * (r.x >> 2);
                    const R wA = q[0], wD = q[1], aA = q[2], aD = q[3];
                    a1 = role == 0 ? wA : (role == 3 ? R(0) : -(role == 1 ? R(1) - aA : aA) * wA);
                    a2 = role == 3 ? wD : (role == 0 ? R(0) : -(role == 1 ? R(1) - aD : aD) * wD);
                }
                Fx += a1 * tn[4 * r.y] + a2 * tn[4 * r.z];
                Fy += a1 * tn[4 * r.y + 1] + a2 * tn[4 * r.z + 1];
                Fz += a1 * tn[4 * r.y + 2] + a2 * tn[4 * r.z + 2];
            }
        }
        // local area (-kal dS/S w), global area (-kag dSg/Sg w), volume
        // (-kv dV/V0 S n_out / 3); w = centroid -> vertex over its length, or
        // (conservative model) over the RMS length of the triangle's three
#pragma unroll 2
        for (int k = o0.z; k < o1.z; ++k) {
            const int4 r = gld(T->t_inc + k);
            const int t = r.x;
            const double gx = (px + xs[3 * r.y] + xs[3 * r.z]) * (1.0 / 3.0);
            const double gy = (py + xs[3 * r.y + 1] + xs[3 * r.z + 1]) * (1.0 / 3.0);
            const double gz = (pz + xs[3 * r.y + 2] + xs[3 * r.z + 2]) * (1.0 / 3.0);
            const R wx = (R)(px - gx), wy = (R)(py - gy), wz = (R)(pz - gz);
            R n2 = wx * wx + wy * wy + wz * wz;
            if (cons) {
                const R bx = (R)(xs[3 * r.y] - gx), by = (R)(xs[3 * r.y + 1] - gy), bz = (R)(xs[3 * r.y + 2] - gz);
                const R qx = (R)(xs[3 * r.z] - gx), qy = (R)(xs[3 * r.z + 1] - gy), qz = (R)(xs[3 * r.z + 2] - gz);
                n2 = (n2 + bx * bx + by * by + bz * bz + qx * qx + qy * qy + qz * qz) * third;
            }
            const R ct = (-kal * tr[t] + cg) / sqrt(n2);
            const R vf = cv * tn[4 * t + 3] * third;
            Fx += ct * wx - vf * tn[4 * t];
            Fy += ct * wy - vf * tn[4 * t + 1];
            Fz += ct * wz - vf * tn[4 * t + 2];
        }

        fs[3 * i] = Fx;
        fs[3 * i + 1] = Fy;
        fs[3 * i + 2] = Fz;
        // lower corner of the node's 2x2x2 stencil (unwrapped lattice index);
        // nodes sit at cell centres, so the stencil starts at floor(x - 1/2)
        int b[3];
        if (stencil_corner(px, py, pz, O.anchor, b)) {
            blo[0] = min(blo[0], b[0]); blo[1] = min(blo[1], b[1]); blo[2] = min(blo[2], b[2]);
            bhi[0] = max(bhi[0], b[0]); bhi[1] = max(bhi[1], b[1]); bhi[2] = max(bhi[2], b[2]);
        } else {
            flags |= ST_NONFINITE;  // no stencil for a non-finite or runaway node
        }
    }
    wave_bbox_to_block(blo, bhi, bbox);
    __syncthreads();

    // Coupling phase.  The object's stencil box (unwrapped lattice indices
    // [o, o + e)) is kept in LDS when it fits: one bit per box node marks the
    // nodes some stencil touches, those nodes are numbered compactly, the
    // fluid velocity u = (sum_i n_i e_i + g/2)/rho is computed once per such
    // node, and the reaction forces of all mesh nodes are summed per lattice
    // node in LDS before one global atomic per node and component.
    const int ox = bbox[0], oy = bbox[1], oz = bbox[2];
    const long long exl = (long long)bbox[3] - ox + 2, eyl = (long long)bbox[4] - oy + 2,
                    ezl = (long long)bbox[5] - oz + 2;
    const bool grid = bbox[3] >= bbox[0] && exl * eyl * ezl <= (long long)ucap;
    const int ex = (int)exl, exy = (int)(exl * eyl);
    unsigned* pre = need + lay.nwords;             // exclusive popcount prefix per word
    R* ug = (R*)carea(lay.ug);                   // [ccap][3] velocity at compact nodes
    int* qn = (int*)carea(lay.qn);               // [ccap] lattice index of compact nodes
    typedef typename Acc<P>::T A;
    constexpr int AW = 3 * Acc<P>::WC;           // accumulator words per node
    A* gacc = (A*)carea(lay.gacc);               // [ccap][AW] summed reaction force
    bool compact = false;
    if (grid) {
        const int vol = (int)(exl * eyl * ezl);
        const int nw = (vol + 31) >> 5;
        for (int k = threadIdx.x; k < nw; k += blockDim.x) need[k] = 0u;
        __syncthreads();
        for (int i = threadIdx.x; i < nn; i += blockDim.x) {
            const int v = node_of(i);
            int b[3];
            if (!stencil_corner(stage(3 * v), stage(3 * v + 1), stage(3 * v + 2), O.anchor, b)) continue;
            const int b0 = (b[2] - oz) * exy + (b[1] - oy) * ex + (b[0] - ox);
            // corners in a lane-rotated order: lanes whose nodes share a cell
            // then hit different words in the same instruction
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = (kk + (int)threadIdx.x) & 7;
                const int idx = b0 + (k >> 2) * exy + ((k >> 1) & 1) * ex + (k & 1);
                atomicOr(&need[idx >> 5], 1u << (idx & 31));
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {  // wave 0: exclusive scan of the per-word popcounts
            const int per = (nw + 63) >> 6;
            const int w0 = threadIdx.x * per;
            unsigned s = 0;
            for (int k = w0; k < w0 + per && k < nw; ++k) s += __popc(need[k]);
            unsigned incl = s;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned o = __shfl_up(incl, off, 64);
                if ((int)threadIdx.x >= off) incl += o;
            }
            unsigned run = incl - s;
            for (int k = w0; k < w0 + per && k < nw; ++k) {
                pre[k] = run;
                run += __popc(need[k]);
            }
            if (threadIdx.x == 63) ncomp = (int)incl;
        }
        __syncthreads();
        compact = ncomp <= ccap;  // block-uniform
        if (compact) {
            for (int k = threadIdx.x; k < AW * ncomp; k += blockDim.x) gacc[k] = A(0);
            // lattice index of every touched node, in compact numbering (the
            // box origin wrapped once, box offsets without integer division)
            const int oxw = wrap_mod(ox, nxb), oyw = wrap_mod(oy, nyb);
            const int ozw = B->walls_z ? oz : wrap_mod(oz, nzb);
            const int ey = (int)eyl;
            const float rex = 1.0f / (float)ex, rey = 1.0f / (float)ey;
            for (int idx = threadIdx.x; idx < vol; idx += blockDim.x) {
                const unsigned word = need[idx >> 5];
                if (!((word >> (idx & 31)) & 1u)) continue;
                const int c = (int)(pre[idx >> 5] + __popc(word & ((1u << (idx & 31)) - 1u)));
                int t, dx, dy, dz;
                divmod_small(idx, ex, rex, t, dx);
                divmod_small(t, ey, rey, dz, dy);
                int gx = oxw + dx, gy = oyw + dy, gz = ozw + dz;
                while (gx >= nxb) gx -= nxb;
                while (gy >= nyb) gy -= nyb;
                if (B->walls_z) {
                    if (gz < 0 || gz >= nzb) flags |= ST_CLAMPED;
                    gz = gz < 0 ? 0 : (gz >= nzb ? nzb - 1 : gz);
                } else {
                    while (gz >= nzb) gz -= nzb;
                }
                qn[c] = (gz * nyb + gy) * nxb + gx;
            }
            __syncthreads();
            if (lists) {  // the slots this workgroup adds to, zeroed by it in the next step
                int* qs = O.qsave + ((size_t)parity * kq + (SPLIT ? slice : 0)) * qstride;
                for (int k = threadIdx.x; k < ncomp; k += blockDim.x) gst(qs + 1 + k, qn[k]);
                if (threadIdx.x == 0) gst(qs, ncomp);
            }
            // fluid velocity there: one dense pass, all population loads in flight
            for (int c = threadIdx.x; c < ncomp; c += blockDim.x) {
                const int q = qn[c];
                if (bt && gld(bt + q)) {  // obstacle node: the wall velocity
                    const double* uw = B->wall_u + 3 * gld(bt + q);
                    ug[3 * c] = (R)gld(uw);
                    ug[3 * c + 1] = (R)gld(uw + 1);
                    ug[3 * c + 2] = (R)gld(uw + 2);
                    continue;
                }
                R dd[19];
#pragma unroll
                for (int i = 0; i < 19; ++i)
                    dd[i] = dec<P>(pop_load(pop, i, q), inv);
                R dr = 0;
#pragma unroll
                for (int i = 0; i < 19; ++i) dr += dd[i];
                const R jx = dd[1] - dd[2] + dd[7] - dd[8] + dd[9] - dd[10] + dd[11] - dd[12] + dd[13] - dd[14];
                const R jy = dd[3] - dd[4] + dd[7] - dd[8] - dd[9] + dd[10] + dd[15] - dd[16] + dd[17] - dd[18];
                const R jz = dd[5] - dd[6] + dd[11] - dd[12] - dd[13] + dd[14] + dd[15] - dd[16] - dd[17] + dd[18];
                const R ir = R(1) / (rho0 + dr);
                ug[3 * c] = (jx + R(0.5) * gx_) * ir;
                ug[3 * c + 1] = (jy + R(0.5) * gy_) * ir;
                ug[3 * c + 2] = (jz + R(0.5) * gz_) * ir;
            }
        }
        __syncthreads();
    }
    // corner by corner with lists kept: the lattice kernel clears G[parity]
    // where it reads it in this step
    if (lists && !compact && threadIdx.x == 0) gst(B->gclear + parity, 1u);

    // per mesh node: interpolate, drag, integrate, spread
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
        const int v = node_of(i);
        const double px = stage(3 * v), py = stage(3 * v + 1), pz = stage(3 * v + 2);
        R vx = gld(O.V + 3 * v), vy = gld(O.V + 3 * v + 1), vz = gld(O.V + 3 * v + 2);
        if (O.F) {  // the half-step velocity, as staged
            vx = fmadd(gld(O.F + 3 * v), half_im, vx);
            vy = fmadd(gld(O.F + 3 * v + 1), half_im, vy);
            vz = fmadd(gld(O.F + 3 * v + 2), half_im, vz);
        }
        R dgx = 0, dgy = 0, dgz = 0;
        int sb[3];
        if (stencil_corner(px, py, pz, O.anchor, sb)) {
            const double sx = px - 0.5, sy = py - 0.5, sz = pz - 0.5;
            const R phx = (R)(sx - floor(sx)), phy = (R)(sy - floor(sy)), phz = (R)(sz - floor(sz));
            if (compact) {
                // corners in an order rotated by the node index (the same for
                // any block size): lanes whose nodes share a cell then add to
                // different LDS accumulators in the same instruction; the
                // integer sums do not depend on the order
                const int rot = v & 7;
                const int b0 = (sb[2] - oz) * exy + (sb[1] - oy) * ex + (sb[0] - ox);
                int cr[8];
                R wr[8];
                R ujx = 0, ujy = 0, ujz = 0;
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const int k = (kk + rot) & 7;
                    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
                    wr[kk] = (dx ? phx : R(1) - phx) * (dy ? phy : R(1) - phy) * (dz ? phz : R(1) - phz);
                    const int idx = b0 + dz * exy + dy * ex + dx;
                    const unsigned word = need[idx >> 5];
                    cr[kk] = (int)(pre[idx >> 5] + __popc(word & ((1u << (idx & 31)) - 1u)));
                    ujx += wr[kk] * ug[3 * cr[kk]];
                    ujy += wr[kk] * ug[3 * cr[kk] + 1];
                    ujz += wr[kk] * ug[3 * cr[kk] + 2];
                }
                // eq. dragforce: the fluid receives xi (v - u), the point its opposite
                dgx = xi * (vx - ujx);
                dgy = xi * (vy - ujy);
                dgz = xi * (vz - ujz);
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    if (wr[kk] == R(0)) continue;
                    flags |= acc_add<P>(&gacc[AW * cr[kk]], wr[kk] * dgx, wr[kk] * dgy, wr[kk] * dgz,
                                         B->fp_scale);
                }
            } else {
                // stencil box too large for LDS: per-corner loads and atomics
                int ix = sb[0] % nxb;
                ix += ix < 0 ? nxb : 0;
                int iy = sb[1] % nyb;
                iy += iy < 0 ? nyb : 0;
                const int ix1 = ix + 1 == nxb ? 0 : ix + 1;
                const int iy1 = iy + 1 == nyb ? 0 : iy + 1;
                int iz0, iz1;
                const int izr = sb[2];
                if (B->walls_z) {
                    iz0 = izr < 0 ? 0 : (izr >= nzb ? nzb - 1 : izr);
                    iz1 = izr + 1 < 0 ? 0 : (izr + 1 >= nzb ? nzb - 1 : izr + 1);
                    if (izr < 0 || izr + 1 >= nzb) flags |= ST_CLAMPED;
                } else {
                    iz0 = izr % nzb;
                    iz0 += iz0 < 0 ? nzb : 0;
                    iz1 = iz0 + 1 == nzb ? 0 : iz0 + 1;
                }
                R ujx = 0, ujy = 0, ujz = 0;
#pragma unroll 1
                for (int k = 0; k < 8; ++k) {
                    R dd[19];
                    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
                    const int qk = ((dz ? iz1 : iz0) * nyb + (dy ? iy1 : iy)) * nxb + (dx ? ix1 : ix);
                    const R wk = (dx ? phx : R(1) - phx) * (dy ? phy : R(1) - phy) * (dz ? phz : R(1) - phz);
                    if (bt && gld(bt + qk)) {  // obstacle node: the wall velocity
                        const double* uw = B->wall_u + 3 * gld(bt + qk);
                        ujx += wk * (R)gld(uw);
                        ujy += wk * (R)gld(uw + 1);
                        ujz += wk * (R)gld(uw + 2);
                        continue;
                    }
#pragma unroll
                    for (int j = 0; j < 19; ++j)
                        dd[j] = dec<P>(pop_load(pop, j, qk), inv);
                    R dr = 0;
#pragma unroll
                    for (int j = 0; j < 19; ++j) dr += dd[j];
                    const R jx = dd[1] - dd[2] + dd[7] - dd[8] + dd[9] - dd[10] + dd[11] - dd[12] + dd[13] - dd[14];
                    const R jy = dd[3] - dd[4] + dd[7] - dd[8] - dd[9] + dd[10] + dd[15] - dd[16] + dd[17] - dd[18];
                    const R jz = dd[5] - dd[6] + dd[11] - dd[12] - dd[13] + dd[14] + dd[15] - dd[16] - dd[17] + dd[18];
                    const R ir = R(1) / (rho0 + dr);
                    ujx += wk * ((jx + R(0.5) * gx_) * ir);
                    ujy += wk * ((jy + R(0.5) * gy_) * ir);
                    ujz += wk * ((jz + R(0.5) * gz_) * ir);
                }
                dgx = xi * (vx - ujx);
                dgy = xi * (vy - ujy);
                dgz = xi * (vz - ujz);
#pragma unroll 1
                for (int k = 0; k < 8; ++k) {
                    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
                    const R wk = (dx ? phx : R(1) - phx) * (dy ? phy : R(1) - phy) * (dz ? phz : R(1) - phz);
                    if (wk == R(0)) continue;
                    A av[AW];
                    Acc<P>::convert(wk * dgx, B->fp_scale, av, flags);
                    Acc<P>::convert(wk * dgy, B->fp_scale, av + AW / 3, flags);
                    Acc<P>::convert(wk * dgz, B->fp_scale, av + 2 * AW / 3, flags);
                    const int qk = ((dz ? iz1 : iz0) * nyb + (dy ? iy1 : iy)) * nxb + (dx ? ix1 : ix);
                    if (bt && gld(bt + qk)) continue;  // an obstacle takes no share
                    acc_flush<P>(B, parity, qk, av);
                }
            }
        }
        // eq. newton.  Symplectic Euler: kick with the total force, then
        // drift.  Velocity Verlet: the second half kick (the drift came
        // first), the total force kept for the next step's first half kick.
        R rx = 0, ry = 0, rz = 0;  // soft-sphere repulsion of this step
        if (O.frep) {
            rx = gld(O.frep + 3 * v);
            ry = gld(O.frep + 3 * v + 1);
            rz = gld(O.frep + 3 * v + 2);
        }
        const R ftx = fs[3 * i] - dgx + O.fext[0] + rx;
        const R fty = fs[3 * i + 1] - dgy + O.fext[1] + ry;
        const R ftz = fs[3 * i + 2] - dgz + O.fext[2] + rz;
        if (O.F) {
            vx += ftx * half_im;
            vy += fty * half_im;
            vz += ftz * half_im;
            gst(O.F + 3 * v, ftx);
            gst(O.F + 3 * v + 1, fty);
            gst(O.F + 3 * v + 2, ftz);
        } else {
            vx += ftx * O.inv_mass;
            vy += fty * O.inv_mass;
            vz += ftz * O.inv_mass;
        }
        gst(O.V + 3 * v, vx);
        gst(O.V + 3 * v + 1, vy);
        gst(O.V + 3 * v + 2, vz);
        const double qx = O.F ? px : px + (double)vx, qy = O.F ? py : py + (double)vy,
                     qz = O.F ? pz : pz + (double)vz;
        gst(O.X + 3 * v, qx);
        gst(O.X + 3 * v + 1, qy);
        gst(O.X + 3 * v + 2, qz);
    }
    if (compact) {
        // one global atomic per touched lattice node and accumulator word
        __syncthreads();
        // (one lane per node and word: a wave's atomics cover the consecutive
        // slots of ~21 nodes (FP32 forms) instead of one component of 64 nodes
        // spread over three arrays)
        for (int k = threadIdx.x; k < AW * ncomp; k += blockDim.x) {
            const int c = k / AW, w = k - AW * c;
            const int q = qn[c];
            if (bt && gld(bt + q)) continue;  // an obstacle takes no share
            const A val = gacc[k];
            if (val != A(0)) gatomic_add((A*)B->G[parity] + Acc<P>::SLOT * (size_t)q + w, val);
            if (w == 0) {
                A any = A(0);
#pragma unroll
                for (int u = 0; u < AW; ++u) any |= gacc[AW * c + u];
                if (any != A(0)) gatomic_or(B->mask + (q >> 6), 1ull << (q & 63));
            }
        }
    }
    // split stepping: the stencils of the new positions, for the next step
    if (mark_next)  // (mark_object begins with a barrier: every new position is written)
        mark_object(O.X, SPLIT ? T->order + n0 : nullptr, nn, O.anchor, B, ucap, need, bbox,
                    B->touch[parity ^ 1]);
    if (flags) gatomic_or(B->status, flags);
}

}  // namespace dev
}  // namespace oif
