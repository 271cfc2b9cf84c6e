// lb_device.h -- device routines of the lattice update (paper, Section
// "Method": the D3Q19 propagation/collision update with an external force
// term, eq. lbequation, and the moment definitions of density and velocity),
// shared by the lattice kernel and the persistent batch kernel.
#pragma once

#include "device_common.h"
#include "fixed_point.h"

namespace oif {
namespace dev {

// Coupling force density at node p, read from the step's G (the node's
// slot: three int64 words at 2^-fixed_point_exp in the FP32 forms, 32 bytes;
// three pairs of int64 words at 2^-30 and 2^-80 in the FP64 form, 64 bytes).
// The membrane workgroups zero their slots in the next step; only where one
// of them spread corner by corner (no list of its slots) is the slot cleared
// here.
template <int P, class BP>
__device__ __forceinline__ void take_force(BP __restrict__ B, int p, int parity, bool clear,
                                           typename Prec<P>::R& fx, typename Prec<P>::R& fy,
                                           typename Prec<P>::R& fz) {
    typedef typename Prec<P>::R R;
    if (P == PREC_FP64) {
        long long* G = (long long*)B->G[parity] + 8 * (size_t)p;
        const long long w0 = gld(G), w1 = gld(G + 1), w2 = gld(G + 2), w3 = gld(G + 3), w4 = gld(G + 4),
                        w5 = gld(G + 5);
        fx += (R)fx_value(w0, w1);
        fy += (R)fx_value(w2, w3);
        fz += (R)fx_value(w4, w5);
        if (clear)
            for (int w = 0; w < 6; ++w) gst(G + w, 0ll);
    } else {
        const unsigned o = (unsigned)p * 32u;
        long long* G = (long long*)B->G[parity];
        const double s = B->fp_inv;
        fx += (R)((double)gload(G, o) * s);
        fy += (R)((double)gload(G, o + 8u) * s);
        fz += (R)((double)gload(G, o + 16u) * s);
        if (clear) {
            gstore(G, o, 0ll);
            gstore(G, o + 8u, 0ll);
            gstore(G, o + 16u, 0ll);
        }
    }
}

// e_i . a over the non-zero components of e_i only (i is a compile-time
// constant once the loops are unrolled)
template <typename R>
__device__ __forceinline__ R edot(int i, R ax, R ay, R az) {
    R s = R(0);
    bool any = false;
    if (cx(i)) {
        s = cx(i) > 0 ? ax : -ax;
        any = true;
    }
    if (cy(i)) {
        s = any ? (cy(i) > 0 ? s + ay : s - ay) : (cy(i) > 0 ? ay : -ay);
        any = true;
    }
    if (cz(i)) s = any ? (cz(i) > 0 ? s + az : s - az) : (cz(i) > 0 ? az : -az);
    return s;
}

// Coefficients 3 w_i of the momentum-carrying (odd) equilibrium parts, for
// the axis and the diagonal directions.  In exact arithmetic they are 1/6 and
// 1/12, and sum_i 3 w_i e_i e_i = I makes the collision return the momentum
// it was given.  Rounded separately to the arithmetic type that identity
// would fail by one rounding (6 fl(1/6) = 1 + 3e-8 in FP32), and a
// momentum multiplied by (1 + 3e-8) every step drifts by 3e-8 times the
// number of steps; so the diagonal coefficient is fl(1/12) and the axis one
// 1/2 - 4 fl(1/12), which is exact in binary floating point and keeps
// c_axis + 4 c_diag = 1/2 exactly.
template <typename R>
__device__ __forceinline__ R codd(int i) {
    return i <= 6 ? R(0.5) - R(4) * (R(1) / R(12)) : R(1) / R(12);
}

// BGK collision with Guo forcing of one node's 19 deviations, in place:
// d_i <- (1 - omega) d_i + omega deq_i + S_i with the force density f
// (eq. lbequation with the external force term; density and velocity are the
// moments of the node's populations, the velocity shifted by half the force).
//   deq_i = w_i [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u^2)]
//   S_i   = (1 - 1/(2 tau)) w_i [3 (e_i - u) + 9 (e_i . u) e_i] . F
// Opposite directions share the parts even in e_i and negate the odd ones, so
// they are formed once per pair.  The odd part of deq_i is written
// 3 w_i e_i . (j + F/2), which is rho 3 w_i e_i . u without the division by
// rho and the multiplication back.  Every operation is rounded as written (no
// contraction into fused multiply-adds beyond the explicit ones), so that all
// lattice kernels that inline this function give the same bits node by node.
//
// ACC (FP32 storage): the odd parts, which carry the momentum, are formed in
// FP64 from the exact FP64 sum j of the stored FP32 deviations, and each new
// deviation is rounded to FP32 once.  In FP32 arithmetic the momentum, rebuilt
// from j + F/2 every step (entirely when tau = 1), picks up rounding residuals
// that repeat from step to step: the force adds a near-constant increment to a
// value that sits on the FP32 grid, so the residual of that addition, and of
// the products after it, does not average out.  Over hundreds of steps of a
// body-force driven flow that drift reached 1e-5 of the velocity; with the odd
// parts in FP64 only the final rounding of each stored value remains, whose
// residuals do average out.  The parts even in e_i (density and the
// second-order terms) stay in FP32.
template <typename R, bool ACC, class BP>
__device__ __forceinline__ void collide(BP __restrict__ B, R (&d)[19], R fx, R fy, R fz) {
#pragma clang fp contract(off)
    R drho = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) drho += d[i];
    const R rho = (R)B->rho0 + drho;
    const R ir = R(1) / rho;
    const R om = (R)B->omega, gu = (R)B->guo;
    const R keep = R(1) - om;
    R ax, ay, az;  // j + F/2 (FP32 path)
    double Ax = 0.0, Ay = 0.0, Az = 0.0;  // j + F/2 in FP64 (ACC)
    if (ACC) {
        // pairs of opposite populations first: each difference is exact in
        // FP64, and few FP64 values are live at a time
        Ax = 0.5 * (double)fx;
        Ay = 0.5 * (double)fy;
        Az = 0.5 * (double)fz;
#pragma unroll
        for (int i = 1; i < 19; i += 2) {
            const double q = (double)d[i] - (double)d[i + 1];
            if (cx(i)) Ax = cx(i) > 0 ? Ax + q : Ax - q;
            if (cy(i)) Ay = cy(i) > 0 ? Ay + q : Ay - q;
            if (cz(i)) Az = cz(i) > 0 ? Az + q : Az - q;
        }
        ax = (R)Ax;
        ay = (R)Ay;
        az = (R)Az;
    } else {
        const R jx = d[1] - d[2] + d[7] - d[8] + d[9] - d[10] + d[11] - d[12] + d[13] - d[14];
        const R jy = d[3] - d[4] + d[7] - d[8] - d[9] + d[10] + d[15] - d[16] + d[17] - d[18];
        const R jz = d[5] - d[6] + d[11] - d[12] - d[13] + d[14] + d[15] - d[16] - d[17] + d[18];
        ax = jx + R(0.5) * fx;
        ay = jy + R(0.5) * fy;
        az = jz + R(0.5) * fz;
    }
    const R ux = ax * ir, uy = ay * ir, uz = az * ir;
    const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
    const R uF3 = R(3) * (ux * fx + uy * fy + uz * fz);
    {  // rest population: e = 0
        const R w = wt<R>(0);
        const R deq = w * fmadd(-rho, usq, drho);
        const R src = -(gu * w) * uF3;
        d[0] = fmadd(keep, d[0], fmadd(om, deq, src));
    }
#pragma unroll
    for (int i = 1; i < 19; i += 2) {  // i and its opposite i + 1, e_{i+1} = -e_i
        const R w = wt<R>(i);
        const R eu = edot<R>(i, ux, uy, uz), eF = edot<R>(i, fx, fy, fz);
        const R even = w * fmadd(rho, fmadd(R(4.5) * eu, eu, -usq), drho);
        const R gw = gu * w;
        const R seven = gw * fmadd(R(9) * eu, eF, -uF3);
        if (ACC) {
            // odd part of omega deq_i + S_i in FP64 (the source's odd part, a
            // constant for a constant force, may keep its FP32 rounding: that
            // is a fixed relative error of the force, not a drift)
            const R sodd = (gu * codd<R>(i)) * eF;
            const double odd = fmadd((double)om * codd<double>(i), edot<double>(i, Ax, Ay, Az), (double)sodd);
            const double ev = (double)fmadd(om, even, seven);
            d[i] = fmadd(keep, d[i], (R)(ev + odd));
            d[i + 1] = fmadd(keep, d[i + 1], (R)(ev - odd));
        } else {
            const R c = codd<R>(i);
            const R odd = c * edot<R>(i, ax, ay, az);
            const R sodd = (gu * c) * eF;
            d[i] = fmadd(keep, d[i], fmadd(om, even + odd, seven + sodd));
            d[i + 1] = fmadd(keep, d[i + 1], fmadd(om, even - odd, seven - sodd));
        }
    }
}

// Multiple-relaxation-time collision of one node's 19 deviations, in place
// (the operator of the paper's LB references, in the orthogonal D3Q19 mode
// space).  Mass is kept and the momentum gains F.  The second moment relaxes
// about its equilibrium rho/3 I + rho u u (u = (j + F/2)/rho): with the
// non-equilibrium part N, the post-collision part is
//   N* = gs dev(N) + gb iso(N) + (1+gs)/2 dev(Phi) + (1+gb)/2 iso(Phi),
// Phi = u F + F u, dev/iso the traceless and trace parts.  The populations are
// rebuilt from density, momentum and second moment as w_i [drho + 3 e.j +
// 4.5 (A : e e - tr A / 3)], A the second moment of the deviations less
// drho/3 I; what that leaves of the incoming populations (the
// non-hydrodynamic part) is kept scaled by g_odd and g_even in its parts odd
// and even under e -> -e.  Rounded as written, like collide(), and, with ACC,
// with the odd (momentum-carrying) parts in FP64 from the exact FP64 momentum
// for the reason given there.
template <typename R, bool ACC, class BP>
__device__ __forceinline__ void collide_mrt(BP __restrict__ B, R (&d)[19], R fx, R fy, R fz) {
#pragma clang fp contract(off)
    R drho = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) drho += d[i];
    R jx, jy, jz;
    double Jx = 0.0, Jy = 0.0, Jz = 0.0;  // the momentum in FP64 (ACC)
    if (ACC) {
#pragma unroll
        for (int i = 1; i < 19; i += 2) {
            const double q = (double)d[i] - (double)d[i + 1];
            if (cx(i)) Jx = cx(i) > 0 ? Jx + q : Jx - q;
            if (cy(i)) Jy = cy(i) > 0 ? Jy + q : Jy - q;
            if (cz(i)) Jz = cz(i) > 0 ? Jz + q : Jz - q;
        }
        jx = (R)Jx;
        jy = (R)Jy;
        jz = (R)Jz;
    } else {
        jx = d[1] - d[2] + d[7] - d[8] + d[9] - d[10] + d[11] - d[12] + d[13] - d[14];
        jy = d[3] - d[4] + d[7] - d[8] - d[9] + d[10] + d[15] - d[16] + d[17] - d[18];
        jz = d[5] - d[6] + d[11] - d[12] - d[13] + d[14] + d[15] - d[16] - d[17] + d[18];
    }
    // second moment of the deviations
    const R sxy = d[7] + d[8] + d[9] + d[10], sxz = d[11] + d[12] + d[13] + d[14];
    const R syz = d[15] + d[16] + d[17] + d[18];
    const R pxx = d[1] + d[2] + sxy + sxz, pyy = d[3] + d[4] + sxy + syz, pzz = d[5] + d[6] + sxz + syz;
    const R pxy = d[7] + d[8] - d[9] - d[10], pxz = d[11] + d[12] - d[13] - d[14];
    const R pyz = d[15] + d[16] - d[17] - d[18];
    const R rho = (R)B->rho0 + drho;
    const R ir = R(1) / rho;
    const R ux = (jx + R(0.5) * fx) * ir;
    const R uy = (jy + R(0.5) * fy) * ir;
    const R uz = (jz + R(0.5) * fz) * ir;
    const R t3 = drho / R(3);
    // A (incoming) and the non-equilibrium stress N = A - rho u u
    const R axx = pxx - t3, ayy = pyy - t3, azz = pzz - t3;
    const R rux = rho * ux, ruy = rho * uy, ruz = rho * uz;
    const R exx = rux * ux, eyy = ruy * uy, ezz = ruz * uz, exy = rux * uy, exz = rux * uz, eyz = ruy * uz;
    const R nxx = axx - exx, nyy = ayy - eyy, nzz = azz - ezz;
    const R nxy = pxy - exy, nxz = pxz - exz, nyz = pyz - eyz;
    const R fxx = R(2) * ux * fx, fyy = R(2) * uy * fy, fzz = R(2) * uz * fz;
    const R fxy = ux * fy + fx * uy, fxz = ux * fz + fx * uz, fyz = uy * fz + fy * uz;
    const R gs = (R)B->gamma_shear, gb = (R)B->gamma_bulk;
    const R hs = R(0.5) * (R(1) + gs), hb = R(0.5) * (R(1) + gb);
    const R trn3 = (nxx + nyy + nzz) / R(3), trf3 = (fxx + fyy + fzz) / R(3);
    const R iso = gb * trn3 + hb * trf3;  // trace part of N*, per diagonal entry
    // post-collision A* = rho u u + N*
    const R bxx = exx + gs * (nxx - trn3) + hs * (fxx - trf3) + iso;
    const R byy = eyy + gs * (nyy - trn3) + hs * (fyy - trf3) + iso;
    const R bzz = ezz + gs * (nzz - trn3) + hs * (fzz - trf3) + iso;
    const R bxy = exy + gs * nxy + hs * fxy, bxz = exz + gs * nxz + hs * fxz, byz = eyz + gs * nyz + hs * fyz;
    const R tra3 = (axx + ayy + azz) / R(3), trb3 = (bxx + byy + bzz) / R(3);
    const R go = (R)B->gamma_odd, ge = (R)B->gamma_even;
    const R kx = jx + fx, ky = jy + fy, kz = jz + fz;  // post-collision momentum
    {  // rest population: even, e = 0
        const R w = wt<R>(0);
        const R hin = w * (drho - R(4.5) * tra3), hout = w * (drho - R(4.5) * trb3);
        d[0] = hout + ge * (d[0] - hin);
    }
#pragma unroll
    for (int i = 1; i < 19; i += 2) {  // i and its opposite i + 1
        const R w = wt<R>(i);
        // A : e e over the non-zero components of e_i
        R qa = R(0), qb = R(0);
        if (cx(i)) { qa = qa + axx; qb = qb + bxx; }
        if (cy(i)) { qa = qa + ayy; qb = qb + byy; }
        if (cz(i)) { qa = qa + azz; qb = qb + bzz; }
        if (cx(i) && cy(i)) { qa = qa + R(2 * cx(i) * cy(i)) * pxy; qb = qb + R(2 * cx(i) * cy(i)) * bxy; }
        if (cx(i) && cz(i)) { qa = qa + R(2 * cx(i) * cz(i)) * pxz; qb = qb + R(2 * cx(i) * cz(i)) * bxz; }
        if (cy(i) && cz(i)) { qa = qa + R(2 * cy(i) * cz(i)) * pyz; qb = qb + R(2 * cy(i) * cz(i)) * byz; }
        const R ein = w * (drho + R(4.5) * (qa - tra3)), eout = w * (drho + R(4.5) * (qb - trb3));
        const R geven = R(0.5) * (d[i] + d[i + 1]) - ein;
        const R even = eout + ge * geven;
        if (ACC) {
            const double c = codd<double>(i);
            const double oin = c * edot<double>(i, Jx, Jy, Jz);
            const double oout = c * edot<double>(i, Jx + (double)fx, Jy + (double)fy, Jz + (double)fz);
            const double godd = 0.5 * ((double)d[i] - (double)d[i + 1]) - oin;
            const double odd = oout + (double)go * godd;
            d[i] = (R)((double)even + odd);
            d[i + 1] = (R)((double)even - odd);
        } else {
            const R c = codd<R>(i);
            const R oin = c * edot<R>(i, jx, jy, jz), oout = c * edot<R>(i, kx, ky, kz);
            const R godd = R(0.5) * (d[i] - d[i + 1]) - oin;
            const R odd = oout + go * godd;
            d[i] = even + odd;
            d[i + 1] = even - odd;
        }
    }
}

// Collision at node p (force density f) and push of the 19 post-collision
// deviations to the neighbours (halfway bounce-back at z walls); with
// obstacles (OBST), a push into a solid node (bit i of `links`) returns to p in
// the opposite direction, less 6 w_i rho0 (e_i . u_wall) (bounce-back from a
// moving obstacle).
// NT: non-temporal reads (a value is dead once read, so these reads need not
// displace the values just pushed, which the next step reads); the values are
// the same either way.  A template choice: two branches that differ only in
// the cache hint are merged by the compiler, hint dropped.
template <int P, bool NT, class BP>
__device__ __forceinline__ void load_pops(BP __restrict__ B, int p, int parity,
                                          typename Prec<P>::S (&raw)[19]) {
    typedef typename Prec<P>::S S;
    const gptr<const S> tile = wave_tile((const S*)B->f[parity], p);
    const unsigned lane = (unsigned)(p & 63) * (unsigned)sizeof(S);
    if (NT) {
#pragma unroll
        for (int i = 0; i < 19; ++i)
            raw[i] = __builtin_nontemporal_load(
                (gptr<const S>)((gptr<const char>)tile + lane + 64u * (unsigned)sizeof(S) * i));
    } else {
#pragma unroll
        for (int i = 0; i < 19; ++i) raw[i] = gload(tile, lane + 64u * (unsigned)sizeof(S) * i);
    }
}

template <int P, bool OBST, bool MRT, class BP>
__device__ __forceinline__ void collide_push(BP __restrict__ B, int p,
                                             const typename Prec<P>::S (&raw)[19], typename Prec<P>::R fx,
                                             typename Prec<P>::R fy, typename Prec<P>::R fz, int parity,
                                             unsigned links) {
    typedef typename Prec<P>::S S;
    typedef typename Prec<P>::R R;
    S* __restrict__ dst = (S*)B->f[parity ^ 1];
    const gptr<S> tile = wave_tile(dst, p);
    const unsigned lane = (unsigned)(p & 63) * (unsigned)sizeof(S);
    const float inv = B->st_inv, scale = B->st_scale;

    // an obstacle node is not updated (its link word was loaded beside the
    // populations, so the test costs no extra round trip)
    if (OBST && (links & 1u)) return;
    R d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = dec<P>(raw[i], inv);
    if (MRT) collide_mrt<R, P == PREC_FP32>(B, d, fx, fy, fz);
    else collide<R, P == PREC_FP32>(B, d, fx, fy, fz);

    // neighbour offsets with periodic wrap
    const int nx = B->nx, ny = B->ny, nz = B->nz;
    const int t = B->div_nx ? (int)(__umulhi((unsigned)p, B->div_nx) >> B->sh_nx) : p;
    const int x = p - t * nx;
    const int z = B->div_ny ? (int)(__umulhi((unsigned)t, B->div_ny) >> B->sh_ny) : t;
    const int y = t - z * ny;
    const int plane = nx * ny;
    // wall velocity of the one moving boundary next to this node (if any)
    R wx = R(0), wy = R(0), wz = R(0);
    const unsigned mid = OBST ? (links >> 23) & 255u : 0u;
    if (mid) {
        wx = (R)gld(B->wall_u + 3 * mid);
        wy = (R)gld(B->wall_u + 3 * mid + 1);
        wz = (R)gld(B->wall_u + 3 * mid + 2);
    }
    const int oxm = x ? -1 : nx - 1, oxp = (x < nx - 1) ? 1 : -(nx - 1);
    const int oym = y ? -nx : (ny - 1) * nx, oyp = (y < ny - 1) ? nx : -(ny - 1) * nx;
    const int ozm = z ? -plane : (nz - 1) * plane, ozp = (z < nz - 1) ? plane : -(nz - 1) * plane;
    const bool wlo = B->walls_z && z == 0;
    const bool whi = B->walls_z && z == nz - 1;

#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const R ds = d[i];
        const S out = enc<P>(ds, scale);
        const bool bounce = (cz(i) > 0 && whi) || (cz(i) < 0 && wlo);
        if (bounce) {
            gstore(tile, lane + 64u * (unsigned)sizeof(S) * opp(i), out);
        } else {
            const int off = (cx(i) > 0 ? oxp : (cx(i) < 0 ? oxm : 0)) +
                            (cy(i) > 0 ? oyp : (cy(i) < 0 ? oym : 0)) +
                            (cz(i) > 0 ? ozp : (cz(i) < 0 ? ozm : 0));
            if (OBST && ((links >> i) & 1u)) {
                // the push ends in a solid node: back to p in the opposite
                // direction, with the wall term of a moving neighbour
                S val = out;
                if (links >> 23) {
                    R euw;
                    if (links >> 31) {  // neighbours of several boundaries: this one's
                        const double* uw = B->wall_u + 3 * gld(B->btype + p + off);
                        euw = R(cx(i)) * (R)gld(uw) + R(cy(i)) * (R)gld(uw + 1) + R(cz(i)) * (R)gld(uw + 2);
                    } else {
                        euw = R(cx(i)) * wx + R(cy(i)) * wy + R(cz(i)) * wz;
                    }
                    val = enc<P>(ds - R(6) * wt<R>(i) * (R)B->rho0 * euw, scale);
                }
                gstore(tile, lane + 64u * (unsigned)sizeof(S) * opp(i), val);
            } else {
                pop_store(dst, i, p + off, out);
            }
        }
    }
}

// OBST: some box of the launch has obstacles; without it that code is left out.
// ALL: mode is LB_ALL (every node is updated, so the population loads go out
// first and are in flight while the mask word and any coupling force are
// fetched).  MRT: the boxes use the multiple-relaxation-time collision.
// The update of lattice node p of box B (nothing for p >= N), called by whole
// waves whose 64 lanes hold the 64 nodes of one population tile.  BP: a plain
// or a constant-address-space pointer to the box descriptor (the latter keeps
// the descriptor in scalar registers where the compiler cannot tell that from
// a kernel argument).
template <int P, bool OBST, bool ALL, bool MRT, bool NT, class BP>
__device__ __forceinline__ void lb_node(BP __restrict__ B, int p, int parity, int mode) {
    typedef typename Prec<P>::S S;
    typedef typename Prec<P>::R R;
    const int N = B->N;
    if (p >= N) return;
    S raw[19];
    if (ALL) load_pops<P, NT>(B, p, parity, raw);

    // Force density: body force plus the coupling force G where the node's mask
    // bit is set.  Mask and touch words cover exactly one wave's 64 nodes; all
    // lanes load a word before the wave's first lane clears it.
    R fx = (R)B->g[0], fy = (R)B->g[1], fz = (R)B->g[2];
    // whether this step's G is cleared here: always when the membrane kernel
    // does not clear it, else where a workgroup spread corner by corner
    // (uniform; loaded beside the mask word, not after it)
    const unsigned gclear = B->g_by_mesh ? gld(B->gclear + parity) : 1u;
    unsigned long long* mk = B->mask + (p >> 6);
    unsigned long long m = 0ull;
    if (ALL) {
        m = gld(mk);
        if (m && (p & 63) == 0) gst(mk, 0ull);
    } else {
        // split update: the nodes outside every stencil of this step run while
        // the membrane kernel spreads (no coupling force can reach them), the
        // others after it
        unsigned long long* tw = B->touch[parity] + (p >> 6);
        const unsigned long long tb = gld(tw);
        const bool mine = (tb >> (p & 63)) & 1ull;
        if (mode == LB_FREE) {
            if (mine) return;
        } else {
            if (tb == 0ull) return;  // the whole wave is untouched
            m = gld(mk);
            if ((p & 63) == 0) {
                gst(tw, 0ull);
                if (m) gst(mk, 0ull);
            }
            if (!mine) return;
        }
    }
    // obstacles: which of the node's pushes end in a solid node (and whether
    // the node itself is solid, tested once its populations are loaded)
    const unsigned links = (OBST && B->links) ? gld(B->links + p) : 0u;
    if (!ALL) load_pops<P, NT>(B, p, parity, raw);
    if ((m >> (p & 63)) & 1ull) take_force<P>(B, p, parity, gclear != 0u, fx, fy, fz);
    collide_push<P, OBST, MRT>(B, p, raw, fx, fy, fz, parity, links);
}


}  // namespace dev
}  // namespace oif
