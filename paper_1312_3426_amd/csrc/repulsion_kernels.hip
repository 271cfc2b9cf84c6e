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
//               velocity Verlet), their cells (edge >= the largest pair
//               range) and the count per bucket (cells hashed into H buckets);
//   scan        bucket starts (exclusive prefix sum);
//   scatter     node ids into their buckets;
//   order       each bucket sorted by node id, so that every node meets its
//               partners in a fixed order (deterministic sums);
//   force       per node: the pairs in the 27 surrounding cells (minimum-image
//               distance in the periodic directions), then every obstacle
//               shape and the z walls; FP64 arithmetic.
#include <limits.h>

#include "device_common.h"

namespace oif {
namespace {

using namespace dev;

__device__ __forceinline__ int bucket_of(const RepDev& D, int cell) {
    return D.direct ? cell : (int)(((unsigned)cell * 2654435761u) >> (32 - D.log2H));
}

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
        atomicAdd(&D.cnt[bucket_of(D, cell)], 1);
    }
}

// exclusive prefix sum of cnt[0, n) in place; cnt[n] = total; cursor = starts
__global__ void __launch_bounds__(1024) scan_block_kernel(int* __restrict__ cnt, int* __restrict__ bsum, int n) {
    __shared__ int wsum[16];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    const int v = i < n ? cnt[i] : 0;
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
    if (i < n) cnt[i] = before + incl - v;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = before + incl;
}

__global__ void __launch_bounds__(1024) scan_top_kernel(int* __restrict__ bsum, int nb) {
    // one workgroup: every thread scans a contiguous run, then the runs
    __shared__ int run[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int s = 0;
    for (int k = b0; k < b0 + per && k < nb; ++k) s += bsum[k];
    run[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int k = 0; k < 1024; ++k) {
            const int t = run[k];
            run[k] = acc;
            acc += t;
        }
    }
    __syncthreads();
    int acc = run[threadIdx.x];
    for (int k = b0; k < b0 + per && k < nb; ++k) {
        const int t = bsum[k];
        bsum[k] = acc;
        acc += t;
    }
}

__global__ void __launch_bounds__(1024) scan_add_kernel(int* __restrict__ cnt, int* __restrict__ cursor,
                                                        const int* __restrict__ bsum, int n, int total) {
    const int i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n) {
        const int v = cnt[i] + bsum[blockIdx.x];
        cnt[i] = v;
        cursor[i] = v;
    }
    if (i == 0) cnt[n] = total;
}

__global__ void __launch_bounds__(256) rep_scatter_kernel(const RepDev* __restrict__ Dp) {
    const RepDev& D = *Dp;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.M) return;
    const int slot = atomicAdd(&D.cursor[bucket_of(D, D.cell[j])], 1);
    D.list[slot] = j;
}

__global__ void __launch_bounds__(256) rep_order_kernel(const RepDev* __restrict__ Dp) {
    const RepDev& D = *Dp;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= D.H) return;
    const int s0 = D.cnt[b], s1 = D.cnt[b + 1];
    for (int s = s0 + 1; s < s1; ++s) {  // insertion sort, buckets are short
        const int v = D.list[s];
        int t = s - 1;
        while (t >= s0 && D.list[t] > v) {
            D.list[t + 1] = D.list[t];
            --t;
        }
        D.list[t + 1] = v;
    }
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

__device__ __forceinline__ void soft_sphere(const SoftSphereDev& ss, double d, const double dir[3], double f[3]) {
    const double e = d - ss.offset;
    if (!(e > 0.0 && e < ss.cutoff)) return;
    const double m = ss.a * ss.n * pow(e, -(ss.n + 1.0));
    for (int c = 0; c < 3; ++c) f[c] += m * dir[c];
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

template <typename R>
__global__ void __launch_bounds__(256) rep_force_kernel(const RepDev* __restrict__ Dp) {
    const RepDev& D = *Dp;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.M) return;
    const double p[3] = {D.pos[3 * j], D.pos[3 * j + 1], D.pos[3 * j + 2]};
    const int tj = D.type[j];
    const bool pz = !D.walls_z;
    double f[3] = {0.0, 0.0, 0.0};
    if (D.pairs) {
        const int cell = D.cell[j];
        const int cx = cell % D.nc[0], t = cell / D.nc[0], cy = t % D.nc[1], cz = t / D.nc[1];
        int lx, hx, ly, hy, lz, hz;
        offsets(D.nc[0], true, lx, hx);
        offsets(D.nc[1], true, ly, hy);
        offsets(D.nc[2], pz, lz, hz);
        for (int dz = lz; dz <= hz; ++dz) {
            int z = cz + dz;
            if (pz) z = (z + D.nc[2]) % D.nc[2];
            else if (z < 0 || z >= D.nc[2]) continue;
            for (int dy = ly; dy <= hy; ++dy) {
                const int y = (cy + dy + D.nc[1]) % D.nc[1];
                for (int dx = lx; dx <= hx; ++dx) {
                    const int x = (cx + dx + D.nc[0]) % D.nc[0];
                    const int nb = (z * D.nc[1] + y) * D.nc[0] + x;
                    const int b = bucket_of(D, nb);
                    for (int s = D.cnt[b]; s < D.cnt[b + 1]; ++s) {
                        const int k = D.list[s];
                        if (k == j || D.cell[k] != nb) continue;
                        const SoftSphereDev& ss = D.pair[tj][D.type[k]];
                        if (ss.a == 0.0) continue;
                        double r[3];
                        for (int c = 0; c < 3; ++c) {
                            r[c] = p[c] - D.pos[3 * k + c];
                            if (c < 2 || pz) r[c] -= D.L[c] * floor(r[c] / D.L[c] + 0.5);
                        }
                        const double d = sqrt(dot3(r, r));
                        const double dir[3] = {r[0] / d, r[1] / d, r[2] / d};
                        soft_sphere(ss, d, dir, f);
                    }
                }
            }
        }
    }
    const SoftSphereDev& ws = D.wall[tj];
    if (ws.a != 0.0) {
        double q[3];
        for (int c = 0; c < 3; ++c) q[c] = (c < 2 || pz) ? p[c] - D.L[c] * floor(p[c] / D.L[c]) : p[c];
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
    for (int c = 0; c < 3; ++c) out[3 * j + c] = (R)f[c];
}

__global__ void __launch_bounds__(256) fill_int_kernel(int* __restrict__ a, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

template <typename R>
hipError_t launch_rep_t(const RepDev& h, const RepDev* d, const void* objs, int nobj, hipStream_t s) {
    const int M = h.M;
    if (M == 0) return hipSuccess;
    if (h.pairs)
        hipLaunchKernelGGL(fill_int_kernel, dim3((h.H + 1 + 255) / 256), dim3(256), 0, s, h.cnt, h.H + 1, 0);
    hipLaunchKernelGGL((rep_bin_kernel<R>), dim3(nobj), dim3(256), 0, s, (const ObjDev<R>*)objs, d);
    if (h.pairs) {
        const int nb = (h.H + 1023) / 1024;
        hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(1024), 0, s, h.cnt, h.bsum, h.H);
        hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, h.bsum, nb);
        hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, s, h.cnt, h.cursor, (const int*)h.bsum, h.H, M);
        hipLaunchKernelGGL(rep_scatter_kernel, dim3((M + 255) / 256), dim3(256), 0, s, d);
        hipLaunchKernelGGL(rep_order_kernel, dim3((h.H + 255) / 256), dim3(256), 0, s, d);
    }
    hipLaunchKernelGGL((rep_force_kernel<R>), dim3((M + 255) / 256), dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_repulsion(const RepDev& h, const RepDev* d, const void* objs, int nobj, int precision,
                            hipStream_t s) {
    return precision == PREC_FP64 ? launch_rep_t<double>(h, d, objs, nobj, s)
                                  : launch_rep_t<float>(h, d, objs, nobj, s);
}

}  // namespace oif
