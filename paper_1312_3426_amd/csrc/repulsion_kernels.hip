// repulsion_kernels.hip -- soft-sphere repulsion of the mesh nodes (the
// object-object and object-wall collisions of the paper's channel script,
// Section "Implementation details": "inter ... soft-sphere a n cutoff offset"
// between part types and with the channel walls): a (d - offset)^-n for
// offset < d < offset + cutoff, pushing the partners apart.
//
// Per step, before the membrane kernel (which adds the result to each node's
// total force):
//   rep_bin     the positions the membrane kernel takes its forces at (those
//               of the step start, or advanced by the half-step velocity with
//               velocity Verlet) and their cells (a regular grid, edge >= the
//               largest pair range); nodes per cell;
//   scan        cell starts (exclusive prefix sum);
//   scatter     node ids into their cells (in whatever order the atomics
//               hand out the slots);
//   gather      positions (wrapped into the box along periodic axes) and
//               types copied into cell order;
//   force       one thread per node in cell order: the partners in the 27
//               surrounding cells, read as contiguous runs, a neighbour cell
//               across a periodic face shifted by the box length (the minimum
//               image: cells are at least the pair range and the box at least
//               twice it); then every obstacle shape and the z walls; FP64
//               arithmetic, each node's terms summed exactly (fixed_point.h),
//               so the result does not depend on the order of the cells'
//               slots.
#include <limits.h>

#include "device_common.h"
#include "fixed_point.h"

namespace oif {
namespace {

using namespace dev;

__device__ __forceinline__ int cell_coord(const RepDev& D, int a, double x, bool periodic) {
    const double w = periodic ? x - D.L[a] * floor(x / D.L[a]) : x;
    const double q = floor(w / D.hc[a]);
    // also catches a non-finite position (the watchdog reports those)
    if (!(q >= 0.0)) return 0;
    return q >= (double)D.nc[a] ? D.nc[a] - 1 : (int)q;
}

template <typename R>
__global__ void __launch_bounds__(256) rep_bin_kernel(const ObjDev<R>* __restrict__ objs, const RepDev* __restrict__ Dp) {
    const ObjDev<R>& O = objs[blockIdx.x];
    const RepDev& D = *Dp;
    const int nv = O.t->nv;
    const R half_im = R(0.5) * O.inv_mass;
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        const int j = O.node0 + v;
        double p[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int k = 3 * v + c;
            // the same expression as the membrane kernel's staging
            const double x = O.F ? O.X[k] + (double)fmadd(O.F[k], half_im, O.V[k]) : O.X[k];
            p[c] = x + (double)O.anchor[c];
            D.pos[3 * j + c] = p[c];
        }
        if (!D.pairs) continue;
        const int cx = cell_coord(D, 0, p[0], true), cy = cell_coord(D, 1, p[1], true);
        const int cz = cell_coord(D, 2, p[2], !D.walls_z);
        const int cell = (cz * D.nc[1] + cy) * D.nc[0] + cx;
        D.cell[j] = cell;
        atomicAdd(&D.cnt[cell], 1);
    }
}

// exclusive scan of the 1024-thread block's values (wave scans, then the
// wave totals); all threads of the block must call it
__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    return before + incl - v;
}

// The four counts of thread t of a block: cnt[4 (1024 b + t) ...], one 16-byte
// access where all four lie below n (cnt is 16-byte aligned).
__device__ __forceinline__ void load4(const int* cnt, int i, int n, int (&v)[4]) {
    if (i + 3 < n) {
        const int4 q = *(const int4*)(cnt + i);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        for (int k = 0; k < 4; ++k) v[k] = i + k < n ? cnt[i + k] : 0;
    }
}
__device__ __forceinline__ void store4(int* a, int i, int n, const int (&v)[4]) {
    if (i + 3 < n) {
        *(int4*)(a + i) = make_int4(v[0], v[1], v[2], v[3]);
    } else {
        for (int k = 0; k < 4; ++k)
            if (i + k < n) a[i + k] = v[k];
    }
}

// exclusive prefix sum of cnt[0, n) in place, per block of 4096 counts (four
// per thread); the block totals go to bsum
__global__ void __launch_bounds__(1024) scan_block_kernel(int* __restrict__ cnt, int* __restrict__ bsum, int n) {
    __shared__ int wsum[16];
    const int i = 4 * (blockIdx.x * 1024 + threadIdx.x);
    int v[4];
    load4(cnt, i, n, v);
    const int t = v[0] + v[1] + v[2] + v[3];
    int acc = block_exclusive_scan(t, wsum);
    int e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        e[k] = acc;
        acc += v[k];
    }
    store4(cnt, i, n, e);
    if (threadIdx.x == 1023) bsum[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(1024) scan_top_kernel(int* __restrict__ bsum, int nb) {
    // one workgroup: every thread sums a contiguous run, the run sums are
    // scanned across the block, then every thread writes its run's prefixes
    __shared__ int wsum[16];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int s = 0;
    for (int k = b0; k < b0 + per && k < nb; ++k) s += bsum[k];
    int acc = block_exclusive_scan(s, wsum);
    for (int k = b0; k < b0 + per && k < nb; ++k) {
        const int t = bsum[k];
        bsum[k] = acc;
        acc += t;
    }
}

// add the block offsets: cnt = cell starts, cursor = a copy for the scatter;
// cnt[n] = total
__global__ void __launch_bounds__(1024) scan_add_kernel(int* __restrict__ cnt, int* __restrict__ cursor,
                                                        const int* __restrict__ bsum, int n, int total) {
    const int i = 4 * (blockIdx.x * 1024 + threadIdx.x);
    if (i < n) {
        int v[4];
        load4(cnt, i, n, v);
        const int b = bsum[blockIdx.x];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += b;
        store4(cnt, i, n, v);
        store4(cursor, i, n, v);
    }
    if (i == 0) cnt[n] = total;
}

__global__ void __launch_bounds__(256) rep_scatter_kernel(const RepDev* __restrict__ Dp) {
    const RepDev& D = *Dp;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.M) return;
    const int slot = atomicAdd(&D.cursor[D.cell[j]], 1);
    D.list[slot] = j;
}

__global__ void __launch_bounds__(256) rep_gather_kernel(const RepDev* __restrict__ Dp) {
    const RepDev& D = *Dp;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= D.M) return;
    const int j = D.list[s];
    for (int c = 0; c < 3; ++c) {
        const double x = D.pos[3 * j + c];
        D.spos[3 * s + c] = (c < 2 || !D.walls_z) ? x - D.L[c] * floor(x / D.L[c]) : x;
    }
    D.stype[s] = D.type[j];
}

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Distance from x to the surface of a shape and the unit vector from the
// closest surface point to x; false if x is inside (no force then).  For a
// rhomboid the closest point is the nearest of the face interiors (projection
// inside the parallelogram), the edges (clamped projection) and so the
// corners.
__device__ bool shape_distance(const ShapeDev& S, const double x[3], double& dist, double dir[3]) {
    if (S.kind == 1) {
        const double d = dot3(x, S.n) - S.dist;
        if (!(d > 0.0)) return false;
        dist = d;
        for (int c = 0; c < 3; ++c) dir[c] = S.n[c];
        return true;
    }
    double r[3] = {x[0] - S.corner[0], x[1] - S.corner[1], x[2] - S.corner[2]};
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        const double st = dot3(r, S.cof[k]) / S.det;
        inside = inside && st >= 0.0 && st <= 1.0;
    }
    if (inside) return false;
    double best2 = INFINITY, bp[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k) {
        const double* u = S.e[(k + 1) % 3];
        const double* v = S.e[(k + 2) % 3];
        const double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v), den = uu * vv - uv * uv;
        for (int side = 0; side < 2; ++side) {  // the two faces with coordinate k fixed
            double q[3];
            for (int c = 0; c < 3; ++c) q[c] = r[c] - side * S.e[k][c];
            const double qu = dot3(q, u), qv = dot3(q, v);
            const double a = (qu * vv - qv * uv) / den, b = (qv * uu - qu * uv) / den;
            if (a >= 0.0 && a <= 1.0 && b >= 0.0 && b <= 1.0) {
                double p[3], d2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    p[c] = side * S.e[k][c] + a * u[c] + b * v[c];
                    d2 += (r[c] - p[c]) * (r[c] - p[c]);
                }
                if (d2 < best2) {
                    best2 = d2;
                    for (int c = 0; c < 3; ++c) bp[c] = p[c];
                }
            }
        }
        const double ee = dot3(S.e[k], S.e[k]);
        for (int i = 0; i < 4; ++i) {  // the four edges along e_k
            double o[3], q[3];
            for (int c = 0; c < 3; ++c) {
                o[c] = (i & 1) * u[c] + (i >> 1) * v[c];
                q[c] = r[c] - o[c];
            }
            double t = dot3(q, S.e[k]) / ee;
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            double p[3], d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                p[c] = o[c] + t * S.e[k][c];
                d2 += (r[c] - p[c]) * (r[c] - p[c]);
            }
            if (d2 < best2) {
                best2 = d2;
                for (int c = 0; c < 3; ++c) bp[c] = p[c];
            }
        }
    }
    dist = sqrt(best2);
    for (int c = 0; c < 3; ++c) dir[c] = (r[c] - bp[c]) / dist;
    return true;
}

// Exact sum of a node's force terms (three components).
struct ForceSum {
    long long hi[3] = {0, 0, 0}, lo[3] = {0, 0, 0};
    bool ok = true;
    __device__ void add(double fx, double fy, double fz) {
        const double g[3] = {fx, fy, fz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            long long h, l;
            ok = fx_split(g[c], h, l) && ok;
            hi[c] += h;
            lo[c] += l;
        }
    }
};

__device__ __forceinline__ void soft_sphere(const SoftSphereDev& ss, double d, const double dir[3], ForceSum& f) {
    const double e = d - ss.offset;
    if (!(e > 0.0 && e < ss.cutoff)) return;
    const double m = ss.a * ss.n * pow(e, -(ss.n + 1.0));
    f.add(m * dir[0], m * dir[1], m * dir[2]);
}

// neighbour cell offsets along one axis: -1..1, each cell once when the
// periodic axis has fewer than three cells
__device__ __forceinline__ void offsets(int nc, bool periodic, int& lo, int& hi) {
    if (!periodic || nc >= 3) {
        lo = -1;
        hi = 1;
    } else {
        lo = 0;
        hi = nc - 1;
    }
}

// One thread per node; with pair interactions the threads take the nodes in
// cell order (slot s holds node list[s]), so a wave's neighbouring cells are
// shared and each cell's partners are a contiguous run of spos.
template <typename R>
__global__ void __launch_bounds__(256) rep_force_kernel(const RepDev* __restrict__ Dp) {
    const RepDev& D = *Dp;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= D.M) return;
    const int j = D.pairs ? D.list[s] : s;
    const int tj = D.type[j];
    const bool pz = !D.walls_z;
    ForceSum f;
    if (D.pairs) {
        const double p[3] = {D.spos[3 * s], D.spos[3 * s + 1], D.spos[3 * s + 2]};
        const int cell = D.cell[j];
        const int cx = cell % D.nc[0], t = cell / D.nc[0], cy = t % D.nc[1], cz = t / D.nc[1];
        int lx, hx, ly, hy, lz, hz;
        offsets(D.nc[0], true, lx, hx);
        offsets(D.nc[1], true, ly, hy);
        offsets(D.nc[2], pz, lz, hz);
        // an axis with fewer than 3 cells: each cell once, the image by rounding
        const bool round_x = D.nc[0] < 3, round_y = D.nc[1] < 3, round_z = pz && D.nc[2] < 3;
        for (int dz = lz; dz <= hz; ++dz) {
            int z = cz + dz;
            double sz = 0.0;  // shift of the neighbour cell's nodes (periodic image)
            if (pz) {
                if (z < 0) { z += D.nc[2]; sz = -D.L[2]; }
                else if (z >= D.nc[2]) { z -= D.nc[2]; sz = D.L[2]; }
            } else if (z < 0 || z >= D.nc[2]) {
                continue;
            }
            for (int dy = ly; dy <= hy; ++dy) {
                int y = cy + dy;
                double sy = 0.0;
                if (y < 0) { y += D.nc[1]; sy = -D.L[1]; }
                else if (y >= D.nc[1]) { y -= D.nc[1]; sy = D.L[1]; }
                const int row = (z * D.nc[1] + y) * D.nc[0];
                // the cells x - 1 .. x + 1 of a row without a wrap are one
                // contiguous run of slots
                const bool run3 = !round_x && cx > 0 && cx + 1 < D.nc[0];
                for (int dx = run3 ? 0 : lx; dx <= (run3 ? 0 : hx); ++dx) {
                    int x = cx + dx;
                    double sx = 0.0;
                    if (x < 0) { x += D.nc[0]; sx = -D.L[0]; }
                    else if (x >= D.nc[0]) { x -= D.nc[0]; sx = D.L[0]; }
                    const int u0 = run3 ? D.cnt[row + cx - 1] : D.cnt[row + x];
                    const int u1 = run3 ? D.cnt[row + cx + 2] : D.cnt[row + x + 1];
                    for (int u = u0; u < u1; ++u) {
                        if (u == s) continue;
                        double r[3] = {p[0] - (D.spos[3 * u] + sx), p[1] - (D.spos[3 * u + 1] + sy),
                                       p[2] - (D.spos[3 * u + 2] + sz)};
                        if (round_x) r[0] -= D.L[0] * rint(r[0] / D.L[0]);
                        if (round_y) r[1] -= D.L[1] * rint(r[1] / D.L[1]);
                        if (round_z) r[2] -= D.L[2] * rint(r[2] / D.L[2]);
                        const double d2 = dot3(r, r);
                        if (!(d2 < D.range2)) continue;  // beyond every pair range
                        const SoftSphereDev& ss = D.pair[tj][D.stype[u]];
                        if (ss.a == 0.0) continue;
                        const double d = sqrt(d2), id = 1.0 / d;
                        const double dir[3] = {r[0] * id, r[1] * id, r[2] * id};
                        soft_sphere(ss, d, dir, f);
                    }
                }
            }
        }
    }
    const SoftSphereDev& ws = D.wall[tj];
    if (ws.a != 0.0) {
        double q[3];
        for (int c = 0; c < 3; ++c) {
            const double x = D.pos[3 * j + c];
            q[c] = (c < 2 || pz) ? x - D.L[c] * floor(x / D.L[c]) : x;
        }
        for (int k = 0; k < D.n_shape; ++k) {
            double d, dir[3];
            if (shape_distance(D.shape[k], q, d, dir)) soft_sphere(ws, d, dir, f);
        }
        if (D.walls_z) {
            const double up[3] = {0.0, 0.0, 1.0}, down[3] = {0.0, 0.0, -1.0};
            if (q[2] > 0.0) soft_sphere(ws, q[2], up, f);
            if (q[2] < D.L[2]) soft_sphere(ws, D.L[2] - q[2], down, f);
        }
    }
    R* out = (R*)D.frep;
    for (int c = 0; c < 3; ++c) out[3 * j + c] = (R)fx_value(f.hi[c], f.lo[c]);
    if (!f.ok) atomicOr(D.status, ST_OVERFLOW);
}

// a[0, n) = v, four per thread (a 16-byte aligned)
__global__ void __launch_bounds__(256) fill_int_kernel(int* __restrict__ a, int n, int v) {
    const int i = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int f[4] = {v, v, v, v};
    if (i < n) store4(a, i, n, f);
}

template <typename R>
hipError_t launch_rep_t(const RepDev& h, const RepDev* d, const void* objs, int nobj, hipStream_t s) {
    const int M = h.M;
    if (M == 0) return hipSuccess;
    const int gm = (M + 255) / 256;
    if (h.pairs)
        hipLaunchKernelGGL(fill_int_kernel, dim3((h.ncell + 1 + 1023) / 1024), dim3(256), 0, s, h.cnt, h.ncell + 1, 0);
    hipLaunchKernelGGL((rep_bin_kernel<R>), dim3(nobj), dim3(256), 0, s, (const ObjDev<R>*)objs, d);
    if (h.pairs) {
        const int nb = (h.ncell + 4095) / 4096;
        hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(1024), 0, s, h.cnt, h.bsum, h.ncell);
        hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, h.bsum, nb);
        hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, s, h.cnt, h.cursor, (const int*)h.bsum,
                           h.ncell, M);
        hipLaunchKernelGGL(rep_scatter_kernel, dim3(gm), dim3(256), 0, s, d);
        hipLaunchKernelGGL(rep_gather_kernel, dim3(gm), dim3(256), 0, s, d);
    }
    hipLaunchKernelGGL((rep_force_kernel<R>), dim3(gm), dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_repulsion(const RepDev& h, const RepDev* d, const void* objs, int nobj, int precision,
                            hipStream_t s) {
    return precision == PREC_FP64 ? launch_rep_t<double>(h, d, objs, nobj, s)
                                  : launch_rep_t<float>(h, d, objs, nobj, s);
}

}  // namespace oif
