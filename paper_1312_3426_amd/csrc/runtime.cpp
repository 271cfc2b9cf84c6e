// runtime.cpp -- host runtime and C ABI of liboif.so (declared in include/oif.h).
//
// Templates are processed on the host in FP64 (topology, relaxed lengths,
// dihedral angles, triangle areas, total area and volume), objects are placed
// on the host, and everything the step touches lives on the device.  The
// device copy of the mesh state is authoritative while stepping; host edits
// first pull it back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include <mutex>

#include "batch_sched.h"
#include "oif.h"
#include "oif_device.h"

using namespace oif;

// Fixed device memory of the allocation-free diagnostics call
// (oif_diagnostics_noalloc): the FP64 partial sums of the lattice blocks and
// of the objects, then the ten final sums.  Every device the library runs on
// holds one such array until the process ends, shared by all contexts there.
// On the host `scratch` names the symbol only, not device memory: host code
// uses the address looked up once per device (scratch_address), never the
// name.
constexpr long long SCRATCH_DOUBLES = 131072;  // 1 MiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

// Device address of `scratch` on `device`, which must be the current device;
// looked up on the first call for that device and kept.
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
        it = g_scratch_addr.emplace(device, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// templates (paper: template creation; relaxed values)
// ---------------------------------------------------------------------------
// Nodes per workgroup of the split membrane launches (at most; the slices
// halve a mesh until they are this small).
constexpr int SLICE_NODES = 768;

struct Template {
    int nv = 0, nt = 0, ne = 0;
    std::vector<double> x;              // stretched coordinates [nv][3]
    std::vector<int> tri;               // [nt][3]
    std::vector<std::array<int, 4>> hinge;
    std::vector<std::array<int, 2>> hinge_tri;
    std::vector<std::array<int, 2>> edge;
    std::vector<double> L0, theta0, S0;
    std::vector<double> hbar;           // mean relaxed wing height per hinge
    double Sg0 = 0, V0 = 0;
    oif_moduli k{};
    int ucap = 0; // lattice nodes of the largest stencil box an object can span
    int ccap = 0; // touched lattice nodes an object may have (LDS capacity)
    // node slices of the split membrane launches: compact patches of the
    // reference shape (recursive halving along the longest extent)
    int nslice = 1, smax = 0;
    std::vector<int> order, slice_off;
    // nodes, triangles and hinges of each patch's sub-template (set when the
    // template is uploaded)
    std::vector<int> pnv, pnt, pne;
    std::vector<int> e_off, h_off, t_off;
    std::vector<std::array<int, 2>> e_inc;
    std::vector<int> h_inc, t_inc;
};

inline int tmpl_conservative(const Template& T) { return T.k.force_model == OIF_FORCES_CONSERVATIVE ? 1 : 0; }

inline void vsub(const double* a, const double* b, double* r) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
inline void vcross(const double* a, const double* b, double* r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
inline double vdot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// vector area (B - A) x (C - A) / 2 of triangle (a, b, c)
void vec_area(const double* x, int a, int b, int c, double* n) {
    double ab[3], ac[3];
    vsub(&x[3 * b], &x[3 * a], ab);
    vsub(&x[3 * c], &x[3 * a], ac);
    vcross(ab, ac, n);
    n[0] *= 0.5; n[1] *= 0.5; n[2] *= 0.5;
}

// Inner dihedral angle of hinge (A, B, C, D): T1 = (A, B, C), T2 = (D, C, B);
// pi + atan2((n1 x n2) . e, n1 . n2) with e = unit(C - B); pi when flat.
double dihedral(const double* x, int A, int B, int C, int D) {
    double n1[3], n2[3], e[3], m[3];
    vec_area(x, A, B, C, n1);
    vec_area(x, D, C, B, n2);
    const double l1 = std::sqrt(vdot(n1, n1)), l2 = std::sqrt(vdot(n2, n2));
    for (int c = 0; c < 3; ++c) { n1[c] /= l1; n2[c] /= l2; }
    vsub(&x[3 * C], &x[3 * B], e);
    const double le = std::sqrt(vdot(e, e));
    for (int c = 0; c < 3; ++c) e[c] /= le;
    vcross(n1, n2, m);
    return M_PI + std::atan2(vdot(m, e), vdot(n1, n2));
}

int build_template(const double* nodes, int nv, const int32_t* tris, int nt, const double* stretch,
                   const oif_moduli* k, Template& T, std::string& err) {
    if (nv < 4 || nt < 4 || !nodes || !tris) { err = "template needs >= 4 nodes and >= 4 triangles"; return OIF_E_ARG; }
    T = Template();
    T.nv = nv; T.nt = nt;
    T.x.resize(3 * (size_t)nv);
    const double s[3] = {stretch ? stretch[0] : 1.0, stretch ? stretch[1] : 1.0, stretch ? stretch[2] : 1.0};
    for (int v = 0; v < nv; ++v)
        for (int c = 0; c < 3; ++c) {
            const double val = nodes[3 * v + c] * s[c];
            if (!std::isfinite(val)) { err = "non-finite template coordinate"; return OIF_E_ARG; }
            T.x[3 * v + c] = val;
        }
    T.tri.assign(tris, tris + 3 * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
        const int a = T.tri[3 * t], b = T.tri[3 * t + 1], c = T.tri[3 * t + 2];
        if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv || a == b || b == c || a == c) {
            err = "triangle " + std::to_string(t) + " has an invalid node id";
            return OIF_E_MESH;
        }
    }
    // half-edges grouped by undirected key; a closed, consistently oriented
    // manifold has exactly one half-edge each way per edge
    struct Half { int from, to, wing, t; };
    std::map<std::pair<int, int>, std::vector<Half>> groups;
    for (int t = 0; t < nt; ++t)
        for (int s3 = 0; s3 < 3; ++s3) {
            Half h{T.tri[3 * t + s3], T.tri[3 * t + (s3 + 1) % 3], T.tri[3 * t + (s3 + 2) % 3], t};
            groups[{std::min(h.from, h.to), std::max(h.from, h.to)}].push_back(h);
        }
    for (auto& kv : groups) {
        const auto& g = kv.second;
        if (g.size() != 2 || g[0].from == g[1].from) {
            err = "edge (" + std::to_string(kv.first.first) + "," + std::to_string(kv.first.second) +
                  ") is not shared by two oppositely oriented triangles";
            return OIF_E_MESH;
        }
        const Half& t1 = g[0].from < g[0].to ? g[0] : g[1];
        const Half& t2 = g[0].from < g[0].to ? g[1] : g[0];
        T.edge.push_back({kv.first.first, kv.first.second});
        T.hinge.push_back({t1.wing, t1.from, t1.to, t2.wing});
        T.hinge_tri.push_back({t1.t, t2.t});
    }
    T.ne = (int)T.edge.size();
    // relaxed values, FP64
    T.L0.resize(T.ne);
    T.theta0.resize(T.ne);
    for (int e = 0; e < T.ne; ++e) {
        double d[3];
        vsub(&T.x[3 * T.edge[e][1]], &T.x[3 * T.edge[e][0]], d);
        T.L0[e] = std::sqrt(vdot(d, d));
        const auto& h = T.hinge[e];
        T.theta0[e] = dihedral(T.x.data(), h[0], h[1], h[2], h[3]);
        if (!(T.L0[e] > 0) || !std::isfinite(T.theta0[e]) || !(T.theta0[e] > 0)) {
            err = "degenerate edge or hinge in template";
            return OIF_E_MESH;
        }
    }
    T.S0.resize(nt);
    double Sg = 0, V = 0;
    const double* r0 = &T.x[0];
    for (int t = 0; t < nt; ++t) {
        const int a = T.tri[3 * t], b = T.tri[3 * t + 1], c = T.tri[3 * t + 2];
        double n[3];
        vec_area(T.x.data(), a, b, c, n);
        T.S0[t] = std::sqrt(vdot(n, n));
        if (!(T.S0[t] > 0)) { err = "degenerate triangle in template"; return OIF_E_MESH; }
        Sg += T.S0[t];
        double pa[3], pb[3], pc[3], bc[3];
        vsub(&T.x[3 * a], r0, pa);
        vsub(&T.x[3 * b], r0, pb);
        vsub(&T.x[3 * c], r0, pc);
        vcross(pb, pc, bc);
        V -= vdot(pa, bc) / 6.0;
    }
    T.Sg0 = Sg;
    T.V0 = V;
    if (!(V > 0)) {
        err = "enclosed volume is not positive: triangle normals must point into the object";
        return OIF_E_MESH;
    }
    T.k = *k;
    // mean relaxed wing height of each hinge, (S(T1) + S(T2)) / L0: the length
    // scale of the gradient form of the bending energy
    T.hbar.resize(T.ne);
    for (int e = 0; e < T.ne; ++e) T.hbar[e] = (T.S0[T.hinge_tri[e][0]] + T.S0[T.hinge_tri[e][1]]) / T.L0[e];
    // Stencil box of an object: nodes within radius Rb of the centroid span at
    // most ceil(2 Rb) + 2 lattice nodes per axis; two more allow for deformation.
    {
        double c[3] = {0, 0, 0}, rb = 0;
        for (int v = 0; v < nv; ++v)
            for (int a = 0; a < 3; ++a) c[a] += T.x[3 * v + a] / nv;
        for (int v = 0; v < nv; ++v) {
            double d[3];
            vsub(&T.x[3 * v], c, d);
            rb = std::max(rb, std::sqrt(vdot(d, d)));
        }
        const double side = std::ceil(2.0 * rb) + 4.0;
        T.ucap = side * side * side < 1e6 ? (int)(side * side * side) : 1000000;
        // Touched lattice nodes an object may have in LDS: the most any of 64
        // rigid placements of the template (rotations and sub-cell shifts
        // from a fixed sequence) touches, with a quarter more and 64 nodes
        // for deformation.  An object that touches more takes the slower
        // per-corner path of the membrane kernel (same results).
        const int sd = (int)side + 2;
        std::vector<unsigned char> mark((size_t)sd * sd * sd);
        int most = 0;
        unsigned long long st = 0x9e3779b97f4a7c15ull;
        auto unif = [&]() {  // xorshift64*: uniform in [0, 1)
            st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
            return (double)((st * 0x2545f4914f6cdd1dull) >> 11) * (1.0 / 9007199254740992.0);
        };
        for (int trial = 0; trial < 64; ++trial) {
            // uniform random rotation from a unit quaternion
            const double u1 = unif(), u2 = 2 * M_PI * unif(), u3 = 2 * M_PI * unif();
            const double qa = std::sqrt(1 - u1) * std::sin(u2), qb = std::sqrt(1 - u1) * std::cos(u2),
                         qc = std::sqrt(u1) * std::sin(u3), qd = std::sqrt(u1) * std::cos(u3);
            const double R[9] = {1 - 2 * (qc * qc + qd * qd), 2 * (qb * qc - qa * qd), 2 * (qb * qd + qa * qc),
                                 2 * (qb * qc + qa * qd), 1 - 2 * (qb * qb + qd * qd), 2 * (qc * qd - qa * qb),
                                 2 * (qb * qd - qa * qc), 2 * (qc * qd + qa * qb), 1 - 2 * (qb * qb + qc * qc)};
            const double off[3] = {unif(), unif(), unif()};
            std::fill(mark.begin(), mark.end(), 0);
            int cnt = 0;
            for (int v = 0; v < nv; ++v) {
                double d[3];
                vsub(&T.x[3 * v], c, d);
                int lo[3];
                for (int a = 0; a < 3; ++a) {
                    const double y = R[3 * a] * d[0] + R[3 * a + 1] * d[1] + R[3 * a + 2] * d[2];
                    lo[a] = (int)std::floor(y + off[a] + 0.5 * side - 0.5);  // >= 0 by construction
                }
                for (int cr = 0; cr < 8; ++cr) {
                    const size_t q = ((size_t)(lo[2] + (cr >> 2)) * sd + lo[1] + ((cr >> 1) & 1)) * sd + lo[0] + (cr & 1);
                    if (q < mark.size() && !mark[q]) {
                        mark[q] = 1;
                        ++cnt;
                    }
                }
            }
            most = std::max(most, cnt);
        }
        T.ccap = std::min(T.ucap, most + most / 4 + 64);
    }
    // node slices for the split launches: about 768 nodes each (a power of two
    // of them), each half of its parent's nodes along the parent's longest
    // extent, ties broken by node index
    {
        int K = 1;
        while ((long long)K * SLICE_NODES < nv) K *= 2;
        T.nslice = K;
        T.order.resize(nv);
        for (int v = 0; v < nv; ++v) T.order[v] = v;
        T.slice_off.assign(1, 0);
        std::function<void(int, int, int)> halve = [&](int lo, int hi, int k) {
            if (k == 1) {
                T.slice_off.push_back(hi);
                return;
            }
            double mn[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, mx[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
            for (int i = lo; i < hi; ++i)
                for (int a = 0; a < 3; ++a) {
                    mn[a] = std::min(mn[a], T.x[3 * T.order[i] + a]);
                    mx[a] = std::max(mx[a], T.x[3 * T.order[i] + a]);
                }
            int ax = 0;
            for (int a = 1; a < 3; ++a)
                if (mx[a] - mn[a] > mx[ax] - mn[ax]) ax = a;
            std::sort(T.order.begin() + lo, T.order.begin() + hi, [&](int a, int b) {
                const double xa = T.x[3 * a + ax], xb = T.x[3 * b + ax];
                return xa != xb ? xa < xb : a < b;
            });
            const int mid = lo + (hi - lo) / 2;
            halve(lo, mid, k / 2);
            halve(mid, hi, k / 2);
        };
        halve(0, nv, K);
        T.smax = 0;
        for (int sl = 0; sl < K; ++sl) T.smax = std::max(T.smax, T.slice_off[sl + 1] - T.slice_off[sl]);
    }
    // per-node incidence lists (CSR)
    std::vector<std::vector<std::array<int, 2>>> ei(nv);
    std::vector<std::vector<int>> hi(nv), ti(nv);
    for (int e = 0; e < T.ne; ++e) {
        ei[T.edge[e][0]].push_back({T.edge[e][1], e});
        ei[T.edge[e][1]].push_back({T.edge[e][0], e});
        for (int r = 0; r < 4; ++r) hi[T.hinge[e][r]].push_back((e << 2) | r);
    }
    for (int t = 0; t < nt; ++t)
        for (int s3 = 0; s3 < 3; ++s3) ti[T.tri[3 * t + s3]].push_back((t << 2) | s3);
    T.e_off.assign(1, 0); T.h_off.assign(1, 0); T.t_off.assign(1, 0);
    for (int v = 0; v < nv; ++v) {
        for (auto& p : ei[v]) T.e_inc.push_back(p);
        for (int c : hi[v]) T.h_inc.push_back(c);
        for (int c : ti[v]) T.t_inc.push_back(c);
        T.e_off.push_back((int)T.e_inc.size());
        T.h_off.push_back((int)T.h_inc.size());
        T.t_off.push_back((int)T.t_inc.size());
    }
    return OIF_OK;
}

struct Object {
    int tid = 0;
    double mass = 1.0;
    int ptype = 0;
    double fext[3] = {0, 0, 0};
    int anchor[3] = {0, 0, 0};
    long long off = 0; // first node in the concatenated mesh arrays
    int nv = 0;
};

// device buffer helper
struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct oif_ctx {
    oif_lattice_desc d{};
    std::string err;
    hipStream_t own = nullptr, stream = nullptr;
    int N = 0;
    size_t st_size = 0;
    void* f[2] = {nullptr, nullptr};
    bool f_bound = false;  // f[] is caller memory (oif_bind_device_buffers)
    void* G = nullptr;          // coupling force: [N][4] 8-byte words, [2][N][4] once the membrane kernel clears it
    size_t G_bytes = 0;
    unsigned* gclear = nullptr; // [2] corner-by-corner flags (BoxDev::gclear)
    unsigned long long* mask = nullptr;
    unsigned long long* touch[2] = {nullptr, nullptr};
    unsigned* status = nullptr;
    // obstacles: host copy of the boundary ids, wall velocities, device arrays
    std::vector<unsigned char> bt_host;
    std::vector<double> wall_host;
    int n_bnd = 0;
    void* bt_dev = nullptr;
    void* link_dev = nullptr;
    void* wall_dev = nullptr;
    hipStream_t side = nullptr;          // lattice update of untouched nodes
    hipEvent_t ev_mark = nullptr, ev_free = nullptr;
    int overlap = 0;
    bool touch_valid = false;            // touch[parity] matches the current positions
    size_t mark_lds = 0;
    BoxDev box{};
    BoxDev* box_dev = nullptr;
    int parity = 0;
    long long steps = 0;
    size_t max_lds = 65536;

    std::vector<Template> tmpl;
    std::vector<Object> obj;
    long long M = 0;
    std::vector<double> Xh, Vh; // host mesh state (absolute positions), valid when !host_stale
    std::vector<double> Fh;     // velocity Verlet: the force carried into the next step
    int integrator = 0;         // OIF_INTEGRATOR_EULER or OIF_INTEGRATOR_VERLET
    // soft-sphere repulsion: interaction tables, obstacle shapes, cell lists
    SoftSphereDev rep_pair[REP_TYPES][REP_TYPES] = {};
    SoftSphereDev rep_wall[REP_TYPES] = {};
    std::vector<ShapeDev> shapes;
    bool rep_on = false;
    RepDev rep_h{};
    DevBuf rep_desc, rep_pos, rep_cell, rep_cnt, rep_cursor, rep_bsum, rep_list, rep_spos, rep_stype, rep_frep,
        rep_type, rep_shape;
    bool host_stale = false;
    bool mesh_dirty = true;     // device mesh arrays must be rebuilt

    // device mesh
    std::vector<DevBuf> tbufs;  // per-template arrays
    DevBuf tmpl_dev, obj_dev, X_dev, V_dev, F_dev, geo_dev, scratch_dev;
    DevBuf qsave_dev;           // per object: the G slots its workgroups added to (ObjDev::qsave)
    std::vector<unsigned char> obj_host; // ObjDev<real> array as uploaded (sorted)
    int n_lds_obj = 0;          // objects [0, n_lds_obj) use LDS, the rest global scratch
    int n_split_obj = 0;        // the next n_split_obj run split over several workgroups each
    int n_cpl_obj = 0;          // the next n_cpl_obj keep their coupling area in LDS
    size_t lds_need = 0;
    size_t split_need = 0;      // LDS per workgroup of the split launches
    size_t cpl_need = 0;        // LDS for the coupling area of the CPL objects
    DevBuf split_work;          // (object, slice) per workgroup of the split launches
    int n_split_work = 0;
    int any_conservative = 0;   // some template uses the conservative force model

    // launch configuration
    int lb_block = 256, mesh_block = 256, remap = 1;
    int lb_nt = 0;  // population reads of the lattice kernel non-temporal
    int graph_steps = 0;
    hipGraphExec_t gexec = nullptr;
    int g_len = 0;

    // diagnostics
    DevBuf part_dev, diag_out;
    int diag_blocks = 256;
    void* scratch_addr = nullptr;  // device address of this device's `scratch` array
};

// Multiplier and shift that divide any q < 2^31 by d (1 <= d <= 4096):
// q / d = (q * m) >> (32 + s) with s = ceil(log2 d) - 1 and m = floor(2^(32+s) / d) + 1.
// With e = m d - 2^(32+s), 0 < e <= d <= 2^(s+1), the product overshoots q / d
// by q e / (d 2^(32+s)) < 1 / d, less than the distance from q / d to the next
// integer; m < 2^32 because d > 2^s unless d is a power of two (then m = 2^31 + 1).
// d = 1 is marked by m = 0 (the kernel takes the quotient as q).
static void div_magic(int d, unsigned* m, int* s) {
    if (d <= 1) { *m = 0; *s = 0; return; }
    int k = 0;
    while ((1 << k) < d) ++k;
    *s = k - 1;
    *m = (unsigned)(((unsigned long long)1 << (32 + k - 1)) / (unsigned long long)d + 1);
}

// Bytes of one population buffer: 19 values per node in tiles of 64 nodes,
// the node count rounded up to whole tiles.
static size_t pop_bytes(const oif_ctx* c) { return 19 * (((size_t)c->N + 63) & ~(size_t)63) * c->st_size; }
// bytes per lattice node of the coupling force G: three int64 words (FP32
// forms) or three pairs of them (FP64 form), padded to 32 / 64
static size_t g_slot(const oif_ctx* c) { return c->d.precision == OIF_PREC_FP64 ? 64 : 32; }

struct oif_batch {
    std::vector<oif_ctx*> ctx;
    std::string err;
    int precision = 0;
    DevBuf boxes_dev, work_dev, obj_dev;
    std::vector<unsigned char> obj_host;
    int nblocks = 0, nobj = 0, n_lds_obj = 0, n_split_obj = 0, n_cpl_obj = 0;
    size_t split_need = 0;
    DevBuf split_work;  // (object index within the split group, slice)
    int n_split_work = 0;
    size_t p_cpl_need = 0;  // persistent form: coupling area of split and CPL objects
    int any_lists = 0;      // some box has the membrane kernel clear its coupling force
    // the work list holds the boxes grouped by lattice-kernel variant
    // (obstacles, MRT collision): one launch per group
    int var_off[5] = {0, 0, 0, 0, 0};
    size_t lds_need = 0;
    size_t cpl_need = 0;
    int any_conservative = 0;
    int lb_block = 256, mesh_block = 256, remap = 1;
    int lb_nt = 0;
    int graph_steps = 0;
    hipGraphExec_t gexec = nullptr;
    int g_len = 0;
    bool built = false;
    // persistent form: one launch per step over a device task list
    int persistent = 0;
    BatchSched sched{};
    DevBuf sched_dev, p_objs, p_group, p_objbox, p_lbwork, p_boxnmesh, p_ctr;
    int p_grid = 0;
    size_t p_lds = 0;
    int p_chunk_req = 0;  // lattice blocks per task as set (0: chosen at build)
    int p_chunk = 1;
};

namespace {

int fail(oif_ctx* c, int code, const std::string& m) {
    if (c) c->err = m;
    return code;
}

#define HIPCALL(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(ctx, e_ == hipErrorOutOfMemory ? OIF_E_NOMEM : OIF_E_HIP,               \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

bool is_fp64(const oif_ctx* c) { return c->d.precision == OIF_PREC_FP64; }
size_t real_size(int prec) { return prec == OIF_PREC_FP64 ? 8 : 4; }

int dev_alloc(oif_ctx* c, DevBuf& b, size_t n) {
    b.release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&b.p, n);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(c, OIF_E_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    b.n = n;
    return OIF_OK;
}

void drop_graph(oif_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_len = 0;
}

// Pull the device mesh state into Xh/Vh (absolute coordinates).
int pull_mesh(oif_ctx* c) {
    if (!c->host_stale || c->M == 0 || !c->X_dev.p) {
        c->host_stale = false;
        return OIF_OK;
    }
    const size_t n = 3 * (size_t)c->M;
    const bool verlet = c->integrator == OIF_INTEGRATOR_VERLET && c->F_dev.p;
    std::vector<double> xl(n), vl(n), fl(verlet ? n : 0);
    HIPCALL(c, hipMemcpyAsync(xl.data(), c->X_dev.p, n * 8, hipMemcpyDeviceToHost, c->stream));
    if (is_fp64(c)) {
        HIPCALL(c, hipMemcpyAsync(vl.data(), c->V_dev.p, n * 8, hipMemcpyDeviceToHost, c->stream));
        if (verlet) HIPCALL(c, hipMemcpyAsync(fl.data(), c->F_dev.p, n * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCALL(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> vf(n), ff(verlet ? n : 0);
        HIPCALL(c, hipMemcpyAsync(vf.data(), c->V_dev.p, n * 4, hipMemcpyDeviceToHost, c->stream));
        if (verlet) HIPCALL(c, hipMemcpyAsync(ff.data(), c->F_dev.p, n * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCALL(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < n; ++i) vl[i] = vf[i];
        for (size_t i = 0; i < ff.size(); ++i) fl[i] = ff[i];
    }
    if (verlet) c->Fh = fl;
    for (const Object& o : c->obj)
        for (int v = 0; v < o.nv; ++v)
            for (int k = 0; k < 3; ++k) {
                const size_t i = 3 * ((size_t)o.off + v) + k;
                c->Xh[i] = xl[i] + o.anchor[k];
                c->Vh[i] = vl[i];
            }
    c->host_stale = false;
    return OIF_OK;
}

// Cell lists and force buffer of the soft-sphere repulsion (when some
// interaction is set and the box holds mesh nodes): a regular grid of cells
// of at least the largest pair range, coarsened until there are at most 16
// cells per mesh node (at least 4096): cells near the pair range keep the
// candidate partners few, the cap keeps the per-cell arrays small next to
// the lattice.
int setup_repulsion(oif_ctx* c, size_t real_bytes) {
    bool pairs = false, walls = false;
    double rc = 0.0;
    for (int a = 0; a < REP_TYPES; ++a) {
        walls = walls || c->rep_wall[a].a > 0.0;
        for (int b = 0; b < REP_TYPES; ++b)
            if (c->rep_pair[a][b].a > 0.0) {
                pairs = true;
                rc = std::max(rc, c->rep_pair[a][b].cutoff + c->rep_pair[a][b].offset);
            }
    }
    c->rep_on = (pairs || walls) && c->M > 0;
    for (DevBuf* b : {&c->rep_desc, &c->rep_pos, &c->rep_cell, &c->rep_cnt, &c->rep_cursor, &c->rep_bsum,
                      &c->rep_list, &c->rep_spos, &c->rep_stype, &c->rep_frep, &c->rep_type, &c->rep_shape})
        b->release();
    if (!c->rep_on) return OIF_OK;
    RepDev& R = c->rep_h;
    R = RepDev{};
    R.M = (int)c->M;
    R.walls_z = c->d.walls_z ? 1 : 0;
    R.pairs = pairs ? 1 : 0;
    R.range2 = rc * rc;
    const int dims[3] = {c->d.nx, c->d.ny, c->d.nz};
    const long long target = std::max(4096LL, 16LL * (long long)c->M);
    for (int a = 0; a < 3; ++a) {
        R.L[a] = dims[a];
        R.nc[a] = pairs ? std::max(1, (int)std::floor(dims[a] / rc)) : 1;
    }
    while ((long long)R.nc[0] * R.nc[1] * R.nc[2] > target) {  // coarser cells are still correct
        int big = 0;
        for (int a = 1; a < 3; ++a)
            if ((double)R.nc[a] / dims[a] > (double)R.nc[big] / dims[big]) big = a;
        R.nc[big] = std::max(1, R.nc[big] - std::max(1, R.nc[big] / 8));
    }
    R.ncell = R.nc[0] * R.nc[1] * R.nc[2];
    for (int a = 0; a < 3; ++a) R.hc[a] = R.L[a] / R.nc[a];
    std::memcpy(R.pair, c->rep_pair, sizeof(R.pair));
    std::memcpy(R.wall, c->rep_wall, sizeof(R.wall));
    const size_t M = c->M, NC = (size_t)R.ncell;
    int rc_ = 0;
    if ((rc_ = dev_alloc(c, c->rep_pos, 3 * M * sizeof(double))) || (rc_ = dev_alloc(c, c->rep_cell, M * 4)) ||
        (rc_ = dev_alloc(c, c->rep_cnt, (NC + 1) * 4)) || (rc_ = dev_alloc(c, c->rep_cursor, NC * 4)) ||
        (rc_ = dev_alloc(c, c->rep_bsum, (NC / 1024 + 1) * 4)) || (rc_ = dev_alloc(c, c->rep_list, M * 4)) ||
        (rc_ = dev_alloc(c, c->rep_spos, 3 * M * sizeof(double))) || (rc_ = dev_alloc(c, c->rep_stype, M)) ||
        (rc_ = dev_alloc(c, c->rep_frep, 3 * M * real_bytes)) || (rc_ = dev_alloc(c, c->rep_type, M)) ||
        (rc_ = dev_alloc(c, c->rep_shape, (c->shapes.size() + 1) * sizeof(ShapeDev))) ||
        (rc_ = dev_alloc(c, c->rep_desc, sizeof(RepDev))))
        return rc_;
    std::vector<unsigned char> types(M);
    for (const Object& o : c->obj)
        for (int v = 0; v < o.nv; ++v) types[(size_t)o.off + v] = (unsigned char)o.ptype;
    HIPCALL(c, hipMemcpy(c->rep_type.p, types.data(), M, hipMemcpyHostToDevice));
    if (!c->shapes.empty())
        HIPCALL(c, hipMemcpy(c->rep_shape.p, c->shapes.data(), c->shapes.size() * sizeof(ShapeDev),
                             hipMemcpyHostToDevice));
    R.n_shape = (int)c->shapes.size();
    R.shape = (const ShapeDev*)c->rep_shape.p;
    R.type = (const unsigned char*)c->rep_type.p;
    R.pos = (double*)c->rep_pos.p;
    R.cell = (int*)c->rep_cell.p;
    R.cnt = (int*)c->rep_cnt.p;
    R.cursor = (int*)c->rep_cursor.p;
    R.bsum = (int*)c->rep_bsum.p;
    R.list = (int*)c->rep_list.p;
    R.spos = (double*)c->rep_spos.p;
    R.stype = (unsigned char*)c->rep_stype.p;
    R.frep = c->rep_frep.p;
    R.status = c->status;
    HIPCALL(c, hipMemcpy(c->rep_desc.p, &R, sizeof(RepDev), hipMemcpyHostToDevice));
    return OIF_OK;
}

// Device-format arrays of a template, or of one patch's sub-template (split
// membrane launches); hinge and incidence entries hold everything the gather
// needs, so a node's entries are independent loads.
struct TArr {
    int nv = 0, nt = 0, ne = 0;
    std::vector<int> tri;           // [nt][3]
    std::vector<int4> noff;         // [nv + 1] (edge, hinge, triangle) list offsets
    std::vector<int2> einc;         // (neighbour, edge)
    std::vector<int4> hinc;         // (hinge << 2 | role, T1, T2, 0)
    std::vector<int4> tinc;         // (triangle, next vertex, vertex after that, 0)
    std::vector<double> L0;         // [ne]
    std::vector<int4> hv;           // [ne] (A, B, C, D)
    std::vector<double> th, cs0;    // [ne], [ne][2]: theta0; cos, sin of theta0 - pi
    std::vector<double> S0;         // [nt]
    std::vector<double> hbar;       // [ne]
    std::vector<int> order, slice_off;
};

TArr template_arrays(const Template& T) {
    TArr A;
    A.nv = T.nv;
    A.nt = T.nt;
    A.ne = T.ne;
    A.tri = T.tri;
    A.L0 = T.L0;
    A.th = T.theta0;
    A.S0 = T.S0;
    A.hbar = T.hbar;
    A.cs0.resize(2 * (size_t)T.ne);
    for (int e = 0; e < T.ne; ++e) {
        A.cs0[2 * e] = std::cos(T.theta0[e] - M_PI);
        A.cs0[2 * e + 1] = std::sin(T.theta0[e] - M_PI);
    }
    A.hv.resize(T.ne);
    for (int e = 0; e < T.ne; ++e) A.hv[e] = make_int4(T.hinge[e][0], T.hinge[e][1], T.hinge[e][2], T.hinge[e][3]);
    A.noff.resize((size_t)T.nv + 1);
    for (int v = 0; v <= T.nv; ++v) A.noff[v] = make_int4(T.e_off[v], T.h_off[v], T.t_off[v], 0);
    A.einc.resize(T.e_inc.size());
    for (size_t k = 0; k < T.e_inc.size(); ++k) A.einc[k] = make_int2(T.e_inc[k][0], T.e_inc[k][1]);
    A.hinc.resize(T.h_inc.size());
    for (size_t k = 0; k < T.h_inc.size(); ++k) {
        const int e = T.h_inc[k] >> 2;
        A.hinc[k] = make_int4(T.h_inc[k], T.hinge_tri[e][0], T.hinge_tri[e][1], 0);
    }
    A.tinc.resize(T.t_inc.size());
    for (size_t k = 0; k < T.t_inc.size(); ++k) {
        const int t = T.t_inc[k] >> 2, s3 = T.t_inc[k] & 3;
        A.tinc[k] = make_int4(t, T.tri[3 * t + (s3 + 1) % 3], T.tri[3 * t + (s3 + 2) % 3], 0);
    }
    A.order = T.order;
    A.slice_off = T.slice_off;
    return A;
}

// Sub-template of patch k: the patch's nodes first (in slice order), then the
// other nodes its triangles and hinges reach; the triangles and hinges the
// patch nodes' gathers read; incidence lists of the patch nodes only, entry
// for entry those of the template, renumbered (so a node's forces are summed
// in the same order as in the whole template).
TArr patch_arrays(const Template& T, const TArr& A, int k) {
    TArr P;
    std::vector<int> nl(T.nv, -1), tl(T.nt, -1), el(T.ne, -1), tris, edges;
    auto addn = [&](int v) {
        if (nl[v] < 0) {
            nl[v] = (int)P.order.size();
            P.order.push_back(v);
        }
    };
    auto addt = [&](int t) {
        if (tl[t] < 0) {
            tl[t] = (int)tris.size();
            tris.push_back(t);
        }
    };
    auto adde = [&](int e) {
        if (el[e] < 0) {
            el[e] = (int)edges.size();
            edges.push_back(e);
        }
    };
    const int s0 = T.slice_off[k], s1 = T.slice_off[k + 1], np = s1 - s0;
    for (int i = s0; i < s1; ++i) addn(T.order[i]);
    for (int i = 0; i < np; ++i) {
        const int v = P.order[i];
        const int4 o0 = A.noff[v], o1 = A.noff[v + 1];
        for (int q = o0.x; q < o1.x; ++q) adde(A.einc[q].y);
        for (int q = o0.y; q < o1.y; ++q) {
            adde(A.hinc[q].x >> 2);
            addt(A.hinc[q].y);
            addt(A.hinc[q].z);
        }
        for (int q = o0.z; q < o1.z; ++q) addt(A.tinc[q].x);
    }
    for (int t : tris)
        for (int a = 0; a < 3; ++a) addn(A.tri[3 * t + a]);
    for (int e : edges) {
        addn(A.hv[e].x);
        addn(A.hv[e].y);
        addn(A.hv[e].z);
        addn(A.hv[e].w);
    }
    P.nv = (int)P.order.size();
    P.nt = (int)tris.size();
    P.ne = (int)edges.size();
    for (int t : tris) {
        for (int a = 0; a < 3; ++a) P.tri.push_back(nl[A.tri[3 * t + a]]);
        P.S0.push_back(A.S0[t]);
    }
    for (int e : edges) {
        const int4 h = A.hv[e];
        P.hv.push_back(make_int4(nl[h.x], nl[h.y], nl[h.z], nl[h.w]));
        P.L0.push_back(A.L0[e]);
        P.th.push_back(A.th[e]);
        P.cs0.push_back(A.cs0[2 * e]);
        P.cs0.push_back(A.cs0[2 * e + 1]);
        P.hbar.push_back(A.hbar[e]);
    }
    P.noff.resize((size_t)P.nv + 1);
    for (int i = 0; i < P.nv; ++i) {
        P.noff[i] = make_int4((int)P.einc.size(), (int)P.hinc.size(), (int)P.tinc.size(), 0);
        if (i >= np) continue;
        const int v = P.order[i];
        const int4 o0 = A.noff[v], o1 = A.noff[v + 1];
        for (int q = o0.x; q < o1.x; ++q) P.einc.push_back(make_int2(nl[A.einc[q].x], el[A.einc[q].y]));
        for (int q = o0.y; q < o1.y; ++q) {
            const int4 h = A.hinc[q];
            P.hinc.push_back(make_int4((el[h.x >> 2] << 2) | (h.x & 3), tl[h.y], tl[h.z], 0));
        }
        for (int q = o0.z; q < o1.z; ++q) {
            const int4 r = A.tinc[q];
            P.tinc.push_back(make_int4(tl[r.x], nl[r.y], nl[r.z], 0));
        }
    }
    P.noff[P.nv] = make_int4((int)P.einc.size(), (int)P.hinc.size(), (int)P.tinc.size(), 0);
    P.slice_off = {0, np};
    return P;
}

template <typename V>
size_t vbytes(const std::vector<V>& v) {
    return (v.size() * sizeof(V) + 15) & ~(size_t)15;
}

size_t tarr_bytes(const TArr& A) {
    return vbytes(A.tri) + vbytes(A.noff) + vbytes(A.einc) + vbytes(A.hinc) + vbytes(A.tinc) + vbytes(A.L0) +
           vbytes(A.hv) + vbytes(A.th) + vbytes(A.cs0) + vbytes(A.S0) + vbytes(A.hbar) + vbytes(A.order) +
           vbytes(A.slice_off);
}

// Copies A's arrays to host[..] and points D's arrays at dev[..] (the same
// offsets in the device buffer the host image is copied to).
template <typename real>
void tarr_place(const TArr& A, unsigned char* host, unsigned char* dev, TmplDev<real>& D) {
    size_t off = 0;
    auto put = [&](const auto& v) -> const void* {
        if (!v.empty()) std::memcpy(host + off, v.data(), v.size() * sizeof(v[0]));
        const void* p = dev + off;
        off += vbytes(v);
        return p;
    };
    D.nv = A.nv;
    D.nt = A.nt;
    D.ne = A.ne;
    D.tri = (const int*)put(A.tri);
    D.n_off = (const int4*)put(A.noff);
    D.e_inc = (const int2*)put(A.einc);
    D.h_inc = (const int4*)put(A.hinc);
    D.t_inc = (const int4*)put(A.tinc);
    D.L0 = (const double*)put(A.L0);
    D.hinge = (const int4*)put(A.hv);
    D.theta0 = (const double*)put(A.th);
    D.cs0 = (const double2*)put(A.cs0);
    D.S0 = (const double*)put(A.S0);
    D.hbar = (const double*)put(A.hbar);
    D.order = (const int*)put(A.order);
    D.slice_off = (const int*)put(A.slice_off);
}

template <typename real>
void tmpl_scalars(const Template& T, TmplDev<real>& D) {
    D.linear = T.k.stretch_law == OIF_STRETCH_LINEAR;
    D.conservative = tmpl_conservative(T);
    D.Sg0 = T.Sg0;
    D.V0 = T.V0;
    D.ks = T.k.ks;
    D.kb = T.k.kb;
    D.kal = T.k.kal;
    D.kag = T.k.kag;
    D.kv = T.k.kv;
    D.ucap = T.ucap;
    D.ccap = T.ccap;
    D.nslice = T.nslice;
    D.smax = T.smax;
}

// LDS per workgroup of the split launches of template T (the larger of the
// sums launch's positions and the largest patch's layout); none when the
// template has a single slice.
size_t split_need_bytes(int precision, const Template& T) {
    if (T.nslice <= 1 || T.pnv.empty()) return SIZE_MAX;
    size_t need = align16((size_t)T.nv * 3 * sizeof(double));
    for (int k = 0; k < T.nslice; ++k)
        need = std::max(need, mesh_lds_bytes(precision, T.pnv[k], T.pnt[k], T.pne[k], T.ucap, T.ccap,
                                             tmpl_conservative(T)));
    return need;
}

template <typename real>
int upload_mesh_t(oif_ctx* c) {
    // per-template arrays
    for (auto& b : c->tbufs) b.release();
    c->tbufs.assign(c->tmpl.size(), DevBuf());
    std::vector<TmplDev<real>> td(c->tmpl.size());
    for (size_t t = 0; t < c->tmpl.size(); ++t) {
        Template& T = c->tmpl[t];
        const TArr A = template_arrays(T);
        std::vector<TArr> pa;
        if (T.nslice > 1)
            for (int k = 0; k < T.nslice; ++k) pa.push_back(patch_arrays(T, A, k));
        T.pnv.clear();
        T.pnt.clear();
        T.pne.clear();
        for (const TArr& P : pa) {
            T.pnv.push_back(P.nv);
            T.pnt.push_back(P.nt);
            T.pne.push_back(P.ne);
        }
        // one allocation: the template's arrays, each patch's arrays, then the
        // patches' descriptors; sub-arrays 16-byte aligned
        size_t total = 0;
        const size_t off_main = total;
        total += tarr_bytes(A);
        std::vector<size_t> off_p;
        for (const TArr& P : pa) {
            off_p.push_back(total);
            total += tarr_bytes(P);
        }
        const size_t off_subs = total;
        total += pa.size() * sizeof(TmplDev<real>);
        int rc = dev_alloc(c, c->tbufs[t], total);
        if (rc) return rc;
        unsigned char* b = (unsigned char*)c->tbufs[t].p;
        std::vector<unsigned char> host(total, 0);
        TmplDev<real>& D = td[t];
        tarr_place(A, host.data() + off_main, b + off_main, D);
        tmpl_scalars(T, D);
        D.subs = pa.empty() ? nullptr : (const TmplDev<real>*)(b + off_subs);
        for (size_t k = 0; k < pa.size(); ++k) {
            TmplDev<real> S{};
            tarr_place(pa[k], host.data() + off_p[k], b + off_p[k], S);
            tmpl_scalars(T, S);
            S.subs = nullptr;
            std::memcpy(host.data() + off_subs + k * sizeof(TmplDev<real>), &S, sizeof(S));
        }
        HIPCALL(c, hipMemcpy(c->tbufs[t].p, host.data(), total, hipMemcpyHostToDevice));
    }
    int rc = dev_alloc(c, c->tmpl_dev, td.size() * sizeof(TmplDev<real>));
    if (rc) return rc;
    HIPCALL(c, hipMemcpy(c->tmpl_dev.p, td.data(), td.size() * sizeof(TmplDev<real>), hipMemcpyHostToDevice));

    // mesh state (object-local) and per-object descriptors
    const size_t n = 3 * (size_t)c->M;
    std::vector<double> xl(n);
    std::vector<real> vl(n);
    for (const Object& o : c->obj)
        for (int v = 0; v < o.nv; ++v)
            for (int k = 0; k < 3; ++k) {
                const size_t i = 3 * ((size_t)o.off + v) + k;
                xl[i] = c->Xh[i] - o.anchor[k];
                vl[i] = (real)c->Vh[i];
            }
    if ((rc = dev_alloc(c, c->X_dev, n * sizeof(double)))) return rc;
    if ((rc = dev_alloc(c, c->V_dev, n * sizeof(real)))) return rc;
    const bool verlet = c->integrator == OIF_INTEGRATOR_VERLET;
    c->F_dev.release();
    if (verlet) {
        std::vector<real> fl(n);
        for (size_t i = 0; i < n; ++i) fl[i] = (real)c->Fh[i];
        if ((rc = dev_alloc(c, c->F_dev, n * sizeof(real)))) return rc;
        if (n) HIPCALL(c, hipMemcpy(c->F_dev.p, fl.data(), n * sizeof(real), hipMemcpyHostToDevice));
    }
    if ((rc = dev_alloc(c, c->geo_dev, 2 * sizeof(double) * (c->obj.size() + 1)))) return rc;
    HIPCALL(c, hipMemcpy(c->X_dev.p, xl.data(), n * sizeof(double), hipMemcpyHostToDevice));
    HIPCALL(c, hipMemcpy(c->V_dev.p, vl.data(), n * sizeof(real), hipMemcpyHostToDevice));

    // objects in four groups, each launched on its own and sorted largest
    // mesh first: meshes staged in LDS whole; meshes split over several
    // workgroups (positions, slice forces and coupling area in LDS, element
    // arrays in the scratch); meshes in the global scratch whose coupling area
    // fits in LDS; meshes entirely in the scratch
    const size_t budget = c->max_lds;
    std::vector<int> order(c->obj.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto need = [&](int i) {
        const Template& T = c->tmpl[c->obj[i].tid];
        return mesh_lds_bytes(c->d.precision, T.nv, T.nt, T.ne, T.ucap, T.ccap, tmpl_conservative(T));
    };
    auto cpl = [&](int i) {
        const Template& T = c->tmpl[c->obj[i].tid];
        return mesh_cpl_lds_bytes(c->d.precision, T.nv, T.nt, T.ne, T.ucap, T.ccap, tmpl_conservative(T));
    };
    auto split = [&](int i) { return split_need_bytes(c->d.precision, c->tmpl[c->obj[i].tid]); };
    auto group = [&](int i) {
        return need(i) <= budget ? 0 : (split(i) <= budget ? 1 : (cpl(i) <= budget ? 2 : 3));
    };
    // scratch of an object outside LDS: the mesh layout, then the slices' sums
    auto scratch_bytes = [&](int i) {
        const Template& T = c->tmpl[c->obj[i].tid];
        return (need(i) + 16 * (size_t)T.nslice + 16 + 255) & ~(size_t)255;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ga = group(a), gb = group(b);
        if (ga != gb) return ga < gb;
        return c->obj[a].nv > c->obj[b].nv;
    });
    c->n_lds_obj = 0;
    c->n_split_obj = 0;
    c->n_cpl_obj = 0;
    c->lds_need = 0;
    c->split_need = 0;
    c->cpl_need = 0;
    c->any_conservative = 0;
    for (const Template& T : c->tmpl) c->any_conservative |= tmpl_conservative(T);
    c->mark_lds = 16;
    for (const Template& T : c->tmpl) c->mark_lds = std::max(c->mark_lds, (size_t)((T.ucap + 31) / 32) * 4);
    c->mark_lds = std::min<size_t>(c->mark_lds, 49152);  // larger stencil boxes mark corner by corner
    size_t scratch_total = 0;
    for (int i : order) {
        const int g = group(i);
        if (g == 0) {
            ++c->n_lds_obj;
            c->lds_need = std::max(c->lds_need, need(i));
        } else {
            scratch_total += scratch_bytes(i);
            if (g == 1) {
                ++c->n_split_obj;
                c->split_need = std::max(c->split_need, split(i));
            } else if (g == 2) {
                ++c->n_cpl_obj;
                c->cpl_need = std::max(c->cpl_need, cpl(i));
            }
        }
    }
    if ((rc = dev_alloc(c, c->scratch_dev, scratch_total))) return rc;
    // slot lists of G (two step parities, one per slice) and clean force
    // buffers: the lists of the objects as they were are gone
    size_t qtotal = 0;
    for (int i : order) {
        const Template& T = c->tmpl[c->obj[i].tid];
        qtotal += 2 * (size_t)T.nslice * ((size_t)T.ccap + 1);
    }
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipStreamSynchronize(c->side));
    if ((rc = dev_alloc(c, c->qsave_dev, 4 * qtotal + 16))) return rc;
    HIPCALL(c, hipMemset(c->qsave_dev.p, 0, 4 * qtotal + 16));
    HIPCALL(c, hipMemset(c->G, 0, c->G_bytes));
    HIPCALL(c, hipMemset(c->gclear, 0, 2 * sizeof(unsigned)));
    {  // the split launches' workgroups: (object index within the group, slice)
        std::vector<int2> w;
        for (int k = 0; k < c->n_split_obj; ++k) {
            const Template& T = c->tmpl[c->obj[order[c->n_lds_obj + k]].tid];
            for (int sl = 0; sl < T.nslice; ++sl) w.push_back(make_int2(k, sl));
        }
        c->n_split_work = (int)w.size();
        c->split_work.release();
        if (!w.empty()) {
            if ((rc = dev_alloc(c, c->split_work, w.size() * sizeof(int2)))) return rc;
            HIPCALL(c, hipMemcpy(c->split_work.p, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice));
        }
    }
    if ((rc = setup_repulsion(c, sizeof(real)))) return rc;
    std::vector<ObjDev<real>> od(c->obj.size());
    size_t soff = 0, qoff = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const Object& o = c->obj[order[k]];
        ObjDev<real>& D = od[k];
        D.t = (const TmplDev<real>*)c->tmpl_dev.p + o.tid;
        D.box = c->box_dev;
        D.X = (double*)c->X_dev.p + 3 * o.off;
        D.V = (real*)c->V_dev.p + 3 * o.off;
        D.F = verlet ? (real*)c->F_dev.p + 3 * o.off : nullptr;
        D.frep = c->rep_on ? (const real*)c->rep_frep.p + 3 * o.off : nullptr;
        D.node0 = o.off;
        D.geo = (double*)c->geo_dev.p + 2 * order[k];
        for (int a = 0; a < 3; ++a) {
            D.anchor[a] = o.anchor[a];
            D.fext[a] = (real)o.fext[a];
        }
        D.inv_mass = (real)(1.0 / o.mass);
        D.mass = o.mass;
        D.scratch = nullptr;
        D.qsave = (int*)c->qsave_dev.p + qoff;
        {
            const Template& T = c->tmpl[o.tid];
            qoff += 2 * (size_t)T.nslice * ((size_t)T.ccap + 1);
        }
        if ((int)k >= c->n_lds_obj) {
            D.scratch = (unsigned char*)c->scratch_dev.p + soff;
            soff += scratch_bytes(order[k]);
        }
    }
    c->obj_host.assign((unsigned char*)od.data(), (unsigned char*)(od.data() + od.size()));
    if ((rc = dev_alloc(c, c->obj_dev, od.size() * sizeof(ObjDev<real>)))) return rc;
    HIPCALL(c, hipMemcpy(c->obj_dev.p, od.data(), od.size() * sizeof(ObjDev<real>), hipMemcpyHostToDevice));
    // diagnostics partials: lattice blocks + objects
    if ((rc = dev_alloc(c, c->part_dev, 5 * sizeof(double) * (c->diag_blocks + c->obj.size() + 1)))) return rc;
    return OIF_OK;
}

int sync_mesh(oif_ctx* c) {
    if (!c->mesh_dirty) return OIF_OK;
    int rc = pull_mesh(c);
    if (rc) return rc;
    drop_graph(c);
    rc = is_fp64(c) ? upload_mesh_t<double>(c) : upload_mesh_t<float>(c);
    if (rc) return rc;
    c->mesh_dirty = false;
    c->touch_valid = false;
    return OIF_OK;
}

size_t objdev_size(int prec) { return prec == OIF_PREC_FP64 ? sizeof(ObjDev<double>) : sizeof(ObjDev<float>); }

// Events bracketing one step's launches (timing only; any may be null).
struct StepEvents {
    hipEvent_t t0 = nullptr, t_mark = nullptr, t_mesh = nullptr, t_wait = nullptr, t_lb = nullptr;
    hipEvent_t f0 = nullptr, f1 = nullptr;  // on the side stream
};

inline void rec(hipEvent_t e, hipStream_t s) {
    if (e) (void)hipEventRecord(e, s);
}

int enqueue_mesh(oif_ctx* c, int par, hipStream_t s, int mark_next) {
    const size_t osz = objdev_size(c->d.precision);
    if (c->rep_on)
        HIPCALL(c, launch_repulsion(c->rep_h, (const RepDev*)c->rep_desc.p, c->obj_dev.p, (int)c->obj.size(),
                                    c->d.precision, s));
    MeshLaunch ml{};
    ml.block = c->mesh_block;
    ml.parity = par;
    ml.mark_next = mark_next;
    ml.conservative = c->any_conservative;
    ml.precision = c->d.precision;
    ml.stream = s;
    ml.lists = c->box.g_by_mesh;
    if (c->n_lds_obj > 0) {
        ml.objs = c->obj_dev.p;
        ml.nobj = c->n_lds_obj;
        ml.lds_bytes = c->lds_need;
        HIPCALL(c, launch_mesh(ml));
    }
    if (c->n_split_obj > 0) {
        MeshLaunch sl = ml;
        sl.objs = (const unsigned char*)c->obj_dev.p + osz * c->n_lds_obj;
        sl.nobj = c->n_split_obj;
        sl.lds_bytes = 0;
        sl.work = (const int2*)c->split_work.p;
        sl.nwork = c->n_split_work;
        sl.split_lds = c->split_need;
        HIPCALL(c, launch_mesh(sl));
    }
    if (c->n_cpl_obj > 0) {
        ml.objs = (const unsigned char*)c->obj_dev.p + osz * (c->n_lds_obj + c->n_split_obj);
        ml.nobj = c->n_cpl_obj;
        ml.lds_bytes = 0;
        ml.cpl_lds_bytes = c->cpl_need;
        HIPCALL(c, launch_mesh(ml));
    }
    const int done = c->n_lds_obj + c->n_split_obj + c->n_cpl_obj;
    if ((int)c->obj.size() > done) {
        ml.objs = (const unsigned char*)c->obj_dev.p + osz * done;
        ml.nobj = (int)c->obj.size() - done;
        ml.lds_bytes = 0;
        ml.cpl_lds_bytes = 0;
        HIPCALL(c, launch_mesh(ml));
    }
    return OIF_OK;
}

int enqueue_lb(oif_ctx* c, int par, hipStream_t s, int mode) {
    LbLaunch ll{};
    ll.boxes = c->box_dev;
    ll.work = nullptr;
    ll.nblocks = (c->N + c->lb_block - 1) / c->lb_block;
    ll.block = c->lb_block;
    ll.parity = par;
    ll.remap = c->remap;
    ll.precision = c->d.precision;
    ll.stream = s;
    ll.mode = mode;
    ll.obstacles = c->n_bnd > 0;
    ll.mrt = c->box.mrt;
    ll.nt = c->lb_nt;
    HIPCALL(c, launch_lb(ll));
    return OIF_OK;
}

// Touch bits of the step of parity c->parity from the current positions, when
// the membrane kernel of the previous step did not leave them (first split
// step, mesh written by the host, a step without split).  Never inside a
// captured graph.
int ensure_touch(oif_ctx* c) {
    if (c->touch_valid || !c->overlap || c->obj.empty()) return OIF_OK;
    const size_t nmask = ((size_t)c->N + 63) / 64;
    HIPCALL(c, hipMemsetAsync(c->touch[0], 0, 8 * nmask, c->stream));
    HIPCALL(c, hipMemsetAsync(c->touch[1], 0, 8 * nmask, c->stream));
    HIPCALL(c, launch_mark(c->obj_dev.p, (int)c->obj.size(), c->d.precision, c->mark_lds, c->parity, c->stream));
    c->touch_valid = true;
    return OIF_OK;
}

// One coupled step.  Without objects, or with overlap off: membrane kernel then
// lattice kernel on `s`.  With overlap (split stepping): the lattice update of
// the nodes outside every stencil of this step runs on the side stream while
// the membrane kernel runs on `s` (it also marks the stencils of the new
// positions for the next step); the stencil nodes are updated once both are
// done, since they need the spread coupling force.
int enqueue_one(oif_ctx* c, int par, hipStream_t s, const StepEvents* ev) {
    StepEvents none;
    const StepEvents& E = ev ? *ev : none;
    int rc;
    if (c->obj.empty() || !c->overlap) {
        rec(E.t0, s);
        if (!c->obj.empty() && (rc = enqueue_mesh(c, par, s, 0))) return rc;
        rec(E.t_mesh, s);
        if ((rc = enqueue_lb(c, par, s, LB_ALL))) return rc;
        rec(E.t_lb, s);
        c->touch_valid = false;
        return OIF_OK;
    }
    rec(E.t0, s);
    rec(E.t_mark, s);
    HIPCALL(c, hipEventRecord(c->ev_mark, s));
    HIPCALL(c, hipStreamWaitEvent(c->side, c->ev_mark, 0));
    rec(E.f0, c->side);
    if ((rc = enqueue_lb(c, par, c->side, LB_FREE))) return rc;
    rec(E.f1, c->side);
    HIPCALL(c, hipEventRecord(c->ev_free, c->side));
    if ((rc = enqueue_mesh(c, par, s, 1))) return rc;
    rec(E.t_mesh, s);
    HIPCALL(c, hipStreamWaitEvent(s, c->ev_free, 0));
    rec(E.t_wait, s);
    if ((rc = enqueue_lb(c, par, s, LB_TOUCHED))) return rc;
    rec(E.t_lb, s);
    return OIF_OK;
}

int enqueue_steps(oif_ctx* c, int n, int parity0, hipStream_t s) {
    int par = parity0;
    for (int k = 0; k < n; ++k) {
        int rc = enqueue_one(c, par, s, nullptr);
        if (rc) return rc;
        par ^= 1;
    }
    return OIF_OK;
}

// FP64 sums of the current state: per-block and per-object partials in
// `part` (5 doubles each), the ten totals in `fin`, copied to out[10].
int run_diag_in(oif_ctx* c, double* part, double* fin, double out[10], unsigned* status) {
    HIPCALL(c, launch_diag_lattice(c->box_dev, c->d.precision, c->parity, part, c->diag_blocks, c->stream));
    HIPCALL(c, launch_diag_mesh(c->obj_dev.p, (int)c->obj.size(), c->d.precision, part + 5 * c->diag_blocks, c->stream));
    HIPCALL(c, launch_diag_final(part, c->diag_blocks, (int)c->obj.size(), fin, c->stream));
    HIPCALL(c, hipMemcpyAsync(out, fin, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCALL(c, hipMemcpyAsync(status, c->status, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    HIPCALL(c, hipStreamSynchronize(c->stream));
    return OIF_OK;
}

int run_diag(oif_ctx* c, double out[10], unsigned* status) {
    return run_diag_in(c, (double*)c->part_dev.p, (double*)c->diag_out.p, out, status);
}

void fill_diag(const oif_ctx* c, const double out[10], unsigned st, oif_diag* d) {
    d->mass = (double)c->N * c->d.rho0 + out[0];
    for (int k = 0; k < 3; ++k) {
        d->momentum_fluid[k] = out[1 + k];
        d->momentum_mesh[k] = out[6 + k];
    }
    d->nonfinite = (out[4] != 0 || out[9] != 0 || (st & ST_NONFINITE)) ? 1 : 0;
    d->clamped = (st & ST_CLAMPED) ? 1 : 0;
    d->overflow = (st & ST_OVERFLOW) ? 1 : 0;
}

int watchdog(oif_ctx* c) {
    double out[10];
    unsigned st = 0;
    int rc = run_diag(c, out, &st);
    if (rc) return rc;
    if (out[4] != 0 || out[9] != 0 || (st & ST_NONFINITE))
        return fail(c, OIF_E_NONFINITE, "watchdog: non-finite populations or mesh state");
    if (st & ST_OVERFLOW) return fail(c, OIF_E_OVERFLOW, "watchdog: coupling force out of fixed-point range");
    return OIF_OK;
}

int check_obj(oif_ctx* c, int oid) {
    if (!c) return OIF_E_ARG;
    if (oid < 0 || oid >= (int)c->obj.size()) return fail(c, OIF_E_ARG, "object id out of range");
    return OIF_OK;
}

int step_impl(oif_ctx* c, int n) {
    int rc = sync_mesh(c);
    if (rc) return rc;
    HIPCALL(c, hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream));
    if ((rc = ensure_touch(c))) return rc;
    int left = n;
    if (c->graph_steps > 0 && n >= c->graph_steps) {
        if (c->parity) {  // the captured graph starts at parity 0
            if ((rc = enqueue_steps(c, 1, c->parity, c->stream))) return rc;
            c->parity ^= 1;
            --left;
        }
        if (!c->gexec || c->g_len != c->graph_steps) {
            drop_graph(c);
            hipGraph_t g = nullptr;
            HIPCALL(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue_steps(c, c->graph_steps, 0, c->stream);
            hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
            HIPCALL(c, e2);
            hipError_t e3 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCALL(c, e3);
            c->g_len = c->graph_steps;
        }
        while (left >= c->graph_steps) {
            HIPCALL(c, hipGraphLaunch(c->gexec, c->stream));
            left -= c->graph_steps;
        }
    }
    if (left > 0) {
        if ((rc = enqueue_steps(c, left, c->parity, c->stream))) return rc;
        c->parity ^= (left & 1);
    }
    c->steps += n;
    if (c->M) c->host_stale = true;
    return watchdog(c);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int oif_lattice_desc_init(oif_lattice_desc* d) {
    if (!d) return OIF_E_ARG;
    std::memset(d, 0, sizeof(*d));
    d->tau = 1.0;
    d->rho0 = 1.0;
    d->precision = OIF_PREC_FP32;
    d->fp16_scale_exp = 12;
    d->fixed_point_exp = 40;
    return OIF_OK;
}

const char* oif_last_error(const oif_ctx* c) { return c ? c->err.c_str() : "null context"; }

int oif_create(const oif_lattice_desc* desc, oif_ctx** out) {
    if (!desc || !out) return OIF_E_ARG;
    *out = nullptr;
    const oif_lattice_desc& d = *desc;
    const long long N = (long long)d.nx * d.ny * d.nz;
    bool ok = d.nx >= 1 && d.ny >= 1 && d.nz >= 1 && d.nx <= 4096 && d.ny <= 4096 && d.nz <= 4096 &&
              (N + 63) / 64 * 64 * 19 < (1LL << 31) && std::isfinite(d.tau) && d.tau > 0.5 && std::isfinite(d.rho0) &&
              d.rho0 > 0 && std::isfinite(d.friction) && d.friction >= 0 && d.precision >= 0 &&
              d.precision <= 3 && d.fp16_scale_exp >= 0 && d.fp16_scale_exp <= 24 &&
              d.fixed_point_exp >= 16 && d.fixed_point_exp <= 56 && (!d.walls_z || d.nz >= 2);
    for (int c = 0; c < 3; ++c) ok = ok && std::isfinite(d.body_force[c]);
    if (!ok) return OIF_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= d.device || d.device < 0) return OIF_E_UNSUPPORTED;
    if (hipSetDevice(d.device) != hipSuccess) return OIF_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, d.device) != hipSuccess) return OIF_E_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return OIF_E_UNSUPPORTED;

    std::unique_ptr<oif_ctx> c(new oif_ctx());
    if (scratch_address(d.device, &c->scratch_addr) != hipSuccess) return OIF_E_HIP;
    c->d = d;
    c->N = (int)N;
    c->st_size = d.precision == OIF_PREC_FP64 ? 8 : (d.precision == OIF_PREC_FP32 ? 4 : 2);
    // non-temporal population reads pay while the two buffers are not much
    // larger than the last-level cache (the autotuner measures both)
    c->lb_nt = 2 * pop_bytes(c.get()) <= ((size_t)1 << 30) ? 1 : 0;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, d.device) == hipSuccess && lds > 0)
        c->max_lds = (size_t)lds;
    // dynamic LDS budget of the membrane kernel: the device's per-workgroup
    // limit minus room for the kernel's static LDS (reduction scratch)
    c->max_lds = c->max_lds > 1024 ? c->max_lds - 1024 : 0;
    if (mesh_set_max_lds(c->max_lds) != hipSuccess) c->max_lds = std::min<size_t>(c->max_lds, 65536 - 1024);
    (void)hipGetLastError();  // the opt-in result must not leak into the next launch check
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_mark, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_free, hipEventDisableTiming) != hipSuccess) {
        oif_destroy(c.release());
        return OIF_E_HIP;
    }
    c->stream = c->own;
    oif_ctx* cp = c.get();
    auto alloc = [&](void** p, size_t n) -> int {
        if (hipMalloc(p, n) != hipSuccess) { *p = nullptr; return OIF_E_NOMEM; }
        return OIF_OK;
    };
    const size_t popb = pop_bytes(cp);
    const size_t nmask = ((size_t)N + 63) / 64;
    int rc = OIF_OK;
    c->G_bytes = g_slot(cp) * (size_t)N;
    if ((rc = alloc(&c->f[0], popb)) || (rc = alloc(&c->f[1], popb)) || (rc = alloc(&c->G, c->G_bytes)) ||
        (rc = alloc((void**)&c->gclear, 2 * sizeof(unsigned))) ||
        (rc = alloc((void**)&c->mask, 8 * nmask)) || (rc = alloc((void**)&c->touch[0], 8 * nmask)) ||
        (rc = alloc((void**)&c->touch[1], 8 * nmask)) ||
        (rc = alloc((void**)&c->status, 256)) ||
        (rc = alloc((void**)&c->box_dev, sizeof(BoxDev)))) {
        oif_destroy(c.release());
        return rc;
    }
    if (hipMemsetAsync(c->f[0], 0, popb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->f[1], 0, popb, c->stream) != hipSuccess ||
        hipMemsetAsync(c->G, 0, c->G_bytes, c->stream) != hipSuccess ||
        hipMemsetAsync(c->gclear, 0, 2 * sizeof(unsigned), c->stream) != hipSuccess ||
        hipMemsetAsync(c->mask, 0, 8 * nmask, c->stream) != hipSuccess ||
        hipMemsetAsync(c->touch[0], 0, 8 * nmask, c->stream) != hipSuccess ||
        hipMemsetAsync(c->touch[1], 0, 8 * nmask, c->stream) != hipSuccess ||
        hipMemsetAsync(c->status, 0, 256, c->stream) != hipSuccess) {
        oif_destroy(c.release());
        return OIF_E_HIP;
    }
    BoxDev& b = c->box;
    b.nx = d.nx; b.ny = d.ny; b.nz = d.nz; b.walls_z = d.walls_z ? 1 : 0;
    b.N = (int)N;
    b.precision = d.precision;
    div_magic(d.nx, &b.div_nx, &b.sh_nx);
    div_magic(d.ny, &b.div_ny, &b.sh_ny);
    b.f[0] = c->f[0]; b.f[1] = c->f[1];
    // the lattice kernel clears G (the default): one buffer for both parities
    b.G[0] = c->G;
    b.G[1] = c->G;
    b.gclear = c->gclear;
    b.g_by_mesh = 0;
    b.mask = c->mask;
    b.touch[0] = c->touch[0];
    b.touch[1] = c->touch[1];
    b.status = c->status;
    for (int k = 0; k < 3; ++k) b.g[k] = d.body_force[k];
    b.rho0 = d.rho0;
    b.omega = 1.0 / d.tau;
    b.guo = 1.0 - 0.5 / d.tau;
    b.xi = d.friction;
    b.st_scale = d.precision == OIF_PREC_FP32_ST_FP16 ? std::ldexp(1.0f, d.fp16_scale_exp) : 1.0f;
    b.st_inv = 1.0f / b.st_scale;
    b.fp_scale = std::ldexp(1.0, d.fixed_point_exp);
    b.fp_inv = std::ldexp(1.0, -d.fixed_point_exp);
    if (hipMemcpyAsync(c->box_dev, &b, sizeof(BoxDev), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        dev_alloc(cp, c->diag_out, 16 * sizeof(double)) != OIF_OK ||
        dev_alloc(cp, c->part_dev, 5 * sizeof(double) * (c->diag_blocks + 1)) != OIF_OK ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        oif_destroy(c.release());
        return OIF_E_HIP;
    }
    *out = c.release();
    return OIF_OK;
}

int oif_destroy(oif_ctx* c) {
    if (!c) return OIF_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->side) (void)hipStreamSynchronize(c->side);
    if (!c->f_bound)
        for (void* p : {c->f[0], c->f[1]})
            if (p) (void)hipFree(p);
    for (void* p : {c->G, (void*)c->gclear, (void*)c->mask, (void*)c->touch[0], (void*)c->touch[1],
                    (void*)c->status, (void*)c->box_dev, c->bt_dev, c->link_dev, c->wall_dev})
        if (p) (void)hipFree(p);
    for (auto& b : c->tbufs) b.release();
    for (DevBuf* b : {&c->tmpl_dev, &c->obj_dev, &c->X_dev, &c->V_dev, &c->F_dev, &c->geo_dev,
                      &c->scratch_dev, &c->split_work, &c->qsave_dev, &c->part_dev, &c->diag_out, &c->rep_desc,
                      &c->rep_pos,
                      &c->rep_cell,
                      &c->rep_cnt, &c->rep_cursor, &c->rep_bsum, &c->rep_list, &c->rep_spos, &c->rep_stype,
                      &c->rep_frep, &c->rep_type, &c->rep_shape})
        b->release();
    if (c->own) (void)hipStreamDestroy(c->own);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_mark) (void)hipEventDestroy(c->ev_mark);
    if (c->ev_free) (void)hipEventDestroy(c->ev_free);
    delete c;
    return OIF_OK;
}

int oif_bind_stream(oif_ctx* c, void* s) {
    if (!c) return OIF_E_ARG;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->stream = s ? (hipStream_t)s : c->own;
    return OIF_OK;
}

int oif_population_bytes(const oif_ctx* c, size_t* bytes) {
    if (!c || !bytes) return OIF_E_ARG;
    *bytes = pop_bytes(c);
    return OIF_OK;
}

int oif_bind_device_buffers(oif_ctx* c, void* f0, void* f1, size_t bytes) {
    if (!c) return OIF_E_ARG;
    if ((f0 == nullptr) != (f1 == nullptr)) return fail(c, OIF_E_ARG, "bind both population buffers or neither");
    const size_t pb = pop_bytes(c);
    if (f0) {
        const uintptr_t a = (uintptr_t)f0, b = (uintptr_t)f1;
        if (bytes < pb) return fail(c, OIF_E_ARG, "population buffers smaller than oif_population_bytes");
        if ((a | b) & 255) return fail(c, OIF_E_ARG, "population buffers must be 256-byte aligned");
        if (a < b + pb && b < a + pb) return fail(c, OIF_E_ARG, "population buffers overlap");
        for (void* p : {f0, f1}) {
            hipPointerAttribute_t at{};
            if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice ||
                at.device != c->d.device) {
                (void)hipGetLastError();
                return fail(c, OIF_E_ARG, "population buffers must be device memory of the context's device");
            }
        }
        // rebinding: a new buffer may be the one it replaces, but no other
        // overlap with the bound ones (the copies would overwrite state)
        if (c->f_bound)
            for (int k = 0; k < 2; ++k)
                for (int j = 0; j < 2; ++j) {
                    const uintptr_t n = k ? b : a, o = (uintptr_t)c->f[j];
                    if (n < o + pb && o < n + pb && !(k == j && n == o))
                        return fail(c, OIF_E_ARG, "population buffers overlap the bound ones other than in place");
                }
    } else if (!c->f_bound) {
        return OIF_OK;  // the context's own buffers already
    }
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipStreamSynchronize(c->side));
    void* nf[2] = {f0, f1};
    if (!f0)  // back to buffers of the context's own
        for (int k = 0; k < 2; ++k)
            if (hipMalloc(&nf[k], pb) != hipSuccess) {
                if (k) (void)hipFree(nf[0]);
                return fail(c, OIF_E_NOMEM, "hipMalloc of the population buffers failed");
            }
    // both buffers carry state (solid nodes keep their values in both)
    for (int k = 0; k < 2; ++k) {
        if (nf[k] == c->f[k]) continue;
        const hipError_t e = hipMemcpy(nf[k], c->f[k], pb, hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
            if (!f0) {
                (void)hipFree(nf[0]);
                (void)hipFree(nf[1]);
            }
            return fail(c, OIF_E_HIP, std::string("copying the populations: ") + hipGetErrorString(e));
        }
    }
    if (!c->f_bound) {
        (void)hipFree(c->f[0]);
        (void)hipFree(c->f[1]);
    }
    c->f[0] = nf[0];
    c->f[1] = nf[1];
    c->f_bound = f0 != nullptr;
    c->box.f[0] = c->f[0];
    c->box.f[1] = c->f[1];
    HIPCALL(c, hipMemcpy(c->box_dev, &c->box, sizeof(BoxDev), hipMemcpyHostToDevice));
    c->mesh_dirty = true;  // batches hold copies of the box descriptor
    drop_graph(c);
    return OIF_OK;
}

int oif_template_create(oif_ctx* c, int tid, const double* nodes, int nv, const int32_t* tris, int nt,
                        const double stretch[3], const oif_moduli* k) {
    if (!c || !k) return OIF_E_ARG;
    if (tid != (int)c->tmpl.size()) return fail(c, OIF_E_ID, "template ids must start at 0 and be consecutive");
    if (!c->obj.empty()) return fail(c, OIF_E_STATE, "templates must be created before objects");
    for (double v : {k->ks, k->kb, k->kal, k->kag, k->kv})
        if (!std::isfinite(v)) return fail(c, OIF_E_ARG, "non-finite modulus");
    if (k->stretch_law != OIF_STRETCH_NEOHOOKE && k->stretch_law != OIF_STRETCH_LINEAR)
        return fail(c, OIF_E_ARG, "unknown stretch law");
    if (k->force_model != OIF_FORCES_PAPER && k->force_model != OIF_FORCES_CONSERVATIVE)
        return fail(c, OIF_E_ARG, "unknown force model");
    if (stretch)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(stretch[a]) || stretch[a] <= 0) return fail(c, OIF_E_ARG, "stretch must be > 0");
    Template T;
    int rc = build_template(nodes, nv, tris, nt, stretch, k, T, c->err);
    if (rc) return rc;
    c->tmpl.push_back(std::move(T));
    c->mesh_dirty = true;
    return OIF_OK;
}

}  // extern "C"

namespace {

// Upload the boundary ids, the per-node bit set of push directions that end
// in a solid node (the built-in z walls act first), and the wall velocities;
// then make both population buffers agree at every node, since nothing streams
// into a solid node and it keeps its values.
int upload_boundaries(oif_ctx* c) {
    HIPCALL(c, hipStreamSynchronize(c->stream));
    for (void** p : {&c->bt_dev, &c->link_dev, &c->wall_dev})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    c->box.btype = nullptr;
    c->box.links = nullptr;
    c->box.wall_u = nullptr;
    if (c->n_bnd > 0) {
        const int nx = c->d.nx, ny = c->d.ny, nz = c->d.nz;
        const std::vector<unsigned char>& bt = c->bt_host;
        std::vector<unsigned> links((size_t)c->N, 0u);
        static const int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        static const int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        static const int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t p = ((size_t)z * ny + y) * nx + x;
                    if (bt[p]) {
                        links[p] = 1u;  // solid
                        continue;
                    }
                    unsigned m = 0;
                    int first = 0;
                    bool several = false, moving = false;
                    for (int i = 1; i < 19; ++i) {
                        int zd = z + ez[i];
                        if (c->d.walls_z && (zd < 0 || zd >= nz)) continue;
                        zd = (zd + nz) % nz;
                        const int xd = (x + ex[i] + nx) % nx, yd = (y + ey[i] + ny) % ny;
                        const unsigned char b = bt[((size_t)zd * ny + yd) * nx + xd];
                        if (!b) continue;
                        m |= 1u << i;
                        if (!first) first = b;
                        several = several || b != first;
                        const double* u = &c->wall_host[3 * b];
                        moving = moving || u[0] != 0.0 || u[1] != 0.0 || u[2] != 0.0;
                    }
                    if (moving) m |= several ? 1u << 31 : (unsigned)first << 23;
                    links[p] = m;
                }
        HIPCALL(c, hipMalloc(&c->bt_dev, (size_t)c->N));
        HIPCALL(c, hipMalloc(&c->link_dev, 4 * (size_t)c->N));
        HIPCALL(c, hipMalloc(&c->wall_dev, 256 * 3 * sizeof(double)));
        HIPCALL(c, hipMemcpy(c->bt_dev, bt.data(), (size_t)c->N, hipMemcpyHostToDevice));
        HIPCALL(c, hipMemcpy(c->link_dev, links.data(), 4 * (size_t)c->N, hipMemcpyHostToDevice));
        HIPCALL(c, hipMemcpy(c->wall_dev, c->wall_host.data(), 256 * 3 * sizeof(double), hipMemcpyHostToDevice));
        c->box.btype = (const unsigned char*)c->bt_dev;
        c->box.links = (const unsigned*)c->link_dev;
        c->box.wall_u = (const double*)c->wall_dev;
    }
    HIPCALL(c, hipMemcpy(c->box_dev, &c->box, sizeof(BoxDev), hipMemcpyHostToDevice));
    HIPCALL(c, hipMemcpy(c->f[c->parity ^ 1], c->f[c->parity], pop_bytes(c), hipMemcpyDeviceToDevice));
    // launches and batches hold copies of the box descriptor: rebuild them
    c->mesh_dirty = true;
    drop_graph(c);
    return OIF_OK;
}

int add_boundary(oif_ctx* c, const double* velocity, int* id, const std::function<bool(double, double, double)>& inside) {
    if (c->n_bnd >= 255) return fail(c, OIF_E_ARG, "at most 255 boundaries");
    if (velocity)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(velocity[k])) return fail(c, OIF_E_ARG, "non-finite boundary velocity");
    if (c->bt_host.empty()) c->bt_host.assign((size_t)c->N, 0);
    if (c->wall_host.empty()) c->wall_host.assign(256 * 3, 0.0);
    const int k = ++c->n_bnd;
    for (int a = 0; a < 3; ++a) c->wall_host[3 * k + a] = velocity ? velocity[a] : 0.0;
    const int nx = c->d.nx, ny = c->d.ny, nz = c->d.nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                if (inside(x + 0.5, y + 0.5, z + 0.5)) c->bt_host[((size_t)z * ny + y) * nx + x] = (unsigned char)k;
    if (id) *id = k;
    return upload_boundaries(c);
}

}  // namespace

extern "C" {

int oif_boundary_rhomboid(oif_ctx* c, const double corner[3], const double a[3], const double b[3],
                          const double cv[3], const double velocity[3], int* id) {
    if (!c || !corner || !a || !b || !cv) return OIF_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(corner[k]) || !std::isfinite(a[k]) || !std::isfinite(b[k]) || !std::isfinite(cv[k]))
            return fail(c, OIF_E_ARG, "non-finite rhomboid");
    double bc[3], ca[3], ab[3];
    vcross(b, cv, bc);
    vcross(cv, a, ca);
    vcross(a, b, ab);
    const double det = vdot(a, bc);
    if (!(std::fabs(det) > 0)) return fail(c, OIF_E_ARG, "degenerate rhomboid");
    const double o[3] = {corner[0], corner[1], corner[2]};
    const double BC[3] = {bc[0], bc[1], bc[2]}, CA[3] = {ca[0], ca[1], ca[2]}, AB[3] = {ab[0], ab[1], ab[2]};
    ShapeDev sh{};
    sh.kind = 0;
    for (int k = 0; k < 3; ++k) {
        sh.corner[k] = corner[k];
        sh.e[0][k] = a[k];
        sh.e[1][k] = b[k];
        sh.e[2][k] = cv[k];
        sh.cof[0][k] = bc[k];
        sh.cof[1][k] = ca[k];
        sh.cof[2][k] = ab[k];
    }
    sh.det = det;
    // the node's coordinates (s, t, u) along a, b, c by Cramer's rule
    const int rc = add_boundary(c, velocity, id, [&](double x, double y, double z) {
        const double r[3] = {x - o[0], y - o[1], z - o[2]};
        const double s = vdot(r, BC) / det, t = vdot(r, CA) / det, u = vdot(r, AB) / det;
        return s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0;
    });
    if (rc == OIF_OK) c->shapes.push_back(sh);  // a refused boundary leaves no shape behind
    return rc;
}

int oif_boundary_wall(oif_ctx* c, const double normal[3], double dist, const double velocity[3], int* id) {
    if (!c || !normal) return OIF_E_ARG;
    const double len = std::sqrt(vdot(normal, normal));
    if (!std::isfinite(dist) || !std::isfinite(len) || !(len > 0)) return fail(c, OIF_E_ARG, "bad wall");
    const double n[3] = {normal[0], normal[1], normal[2]};
    ShapeDev sh{};
    sh.kind = 1;
    for (int k = 0; k < 3; ++k) sh.n[k] = normal[k] / len;
    sh.dist = dist;
    const int rc = add_boundary(c, velocity, id, [&](double x, double y, double z) {
        const double r[3] = {x, y, z};
        return vdot(r, n) / len - dist < 0.0;
    });
    if (rc == OIF_OK) c->shapes.push_back(sh);
    return rc;
}

int oif_boundary_clear(oif_ctx* c) {
    if (!c) return OIF_E_ARG;
    c->n_bnd = 0;
    c->shapes.clear();
    c->bt_host.clear();
    c->wall_host.clear();
    return upload_boundaries(c);
}

int oif_read_boundary(oif_ctx* c, uint8_t* out) {
    if (!c || !out) return OIF_E_ARG;
    if (c->bt_host.empty()) std::memset(out, 0, (size_t)c->N);
    else std::memcpy(out, c->bt_host.data(), (size_t)c->N);
    return OIF_OK;
}

int oif_euler_to_rot(double rx, double ry, double rz, double R[9]) {
    if (!R) return OIF_E_ARG;
    const double cx = std::cos(rx), sx = std::sin(rx), cy = std::cos(ry), sy = std::sin(ry),
                 cz = std::cos(rz), sz = std::sin(rz);
    // Rz * Ry * Rx
    R[0] = cz * cy; R[1] = cz * sy * sx - sz * cx; R[2] = cz * sy * cx + sz * sx;
    R[3] = sz * cy; R[4] = sz * sy * sx + cz * cx; R[5] = sz * sy * cx - cz * sx;
    R[6] = -sy;     R[7] = cy * sx;                R[8] = cy * cx;
    return OIF_OK;
}

int oif_object_add(oif_ctx* c, int oid, int tid, const double origin[3], const double rot[9], double mass,
                   int part_type) {
    if (!c || !origin) return OIF_E_ARG;
    if (oid != (int)c->obj.size()) return fail(c, OIF_E_ID, "object ids must start at 0 and be consecutive");
    if (tid < 0 || tid >= (int)c->tmpl.size()) return fail(c, OIF_E_ARG, "unknown template id");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(origin[a]) || std::fabs(origin[a]) > 1e6) return fail(c, OIF_E_ARG, "origin must be finite, |o| <= 1e6");
    if (rot)
        for (int a = 0; a < 9; ++a)
            if (!std::isfinite(rot[a])) return fail(c, OIF_E_ARG, "non-finite rotation");
    if (!std::isfinite(mass)) return fail(c, OIF_E_ARG, "non-finite mass");
    if (part_type < 0 || part_type >= REP_TYPES) return fail(c, OIF_E_ARG, "part types must lie in 0..15");
    int rc = pull_mesh(c);
    if (rc) return rc;
    const Template& T = c->tmpl[tid];
    Object o;
    o.tid = tid;
    o.mass = mass > 0 ? mass : 1.0;
    o.ptype = part_type;
    o.nv = T.nv;
    o.off = c->M;
    // positions are kept absolute in FP64 (anchor 0): the representation the
    // host reads and writes, so checkpoints round-trip bit for bit
    for (int a = 0; a < 3; ++a) o.anchor[a] = 0;
    const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    const double* R = rot ? rot : I;
    c->Xh.resize(3 * (size_t)(c->M + T.nv));
    c->Vh.resize(3 * (size_t)(c->M + T.nv), 0.0);
    c->Fh.resize(3 * (size_t)(c->M + T.nv), 0.0);
    for (int v = 0; v < T.nv; ++v) {
        const double* p = &T.x[3 * v];
        for (int a = 0; a < 3; ++a)
            c->Xh[3 * ((size_t)o.off + v) + a] = origin[a] + R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2];
    }
    c->M += T.nv;
    c->obj.push_back(o);
    c->mesh_dirty = true;
    return OIF_OK;
}

int oif_object_set_force(oif_ctx* c, int oid, const double f[3]) {
    int rc = check_obj(c, oid);
    if (rc) return rc;
    if (!f || !std::isfinite(f[0]) || !std::isfinite(f[1]) || !std::isfinite(f[2])) return fail(c, OIF_E_ARG, "bad force");
    for (int a = 0; a < 3; ++a) c->obj[oid].fext[a] = f[a];
    c->mesh_dirty = true;
    return OIF_OK;
}

int oif_object_set_origin(oif_ctx* c, int oid, const double o[3]) {
    int rc = check_obj(c, oid);
    if (rc) return rc;
    if (!o) return OIF_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(o[a]) || std::fabs(o[a]) > 1e6) return fail(c, OIF_E_ARG, "origin must be finite, |o| <= 1e6");
    if ((rc = pull_mesh(c))) return rc;
    const Object& ob = c->obj[oid];
    double mean[3] = {0, 0, 0};
    for (int v = 0; v < ob.nv; ++v)
        for (int a = 0; a < 3; ++a) mean[a] += c->Xh[3 * ((size_t)ob.off + v) + a];
    for (int a = 0; a < 3; ++a) mean[a] /= ob.nv;
    for (int v = 0; v < ob.nv; ++v)
        for (int a = 0; a < 3; ++a) c->Xh[3 * ((size_t)ob.off + v) + a] += o[a] - mean[a];
    c->mesh_dirty = true;
    return OIF_OK;
}

int oif_object_set_nodes(oif_ctx* c, int oid, const double* x) {
    return oif_write_mesh(c, oid, x, nullptr);
}

int oif_write_mesh(oif_ctx* c, int oid, const double* X, const double* V) {
    if (!c) return OIF_E_ARG;
    if (oid != -1) {
        int rc = check_obj(c, oid);
        if (rc) return rc;
    }
    int rc = pull_mesh(c);
    if (rc) return rc;
    const size_t off = oid < 0 ? 0 : 3 * (size_t)c->obj[oid].off;
    const size_t n = oid < 0 ? 3 * (size_t)c->M : 3 * (size_t)c->obj[oid].nv;
    for (size_t i = 0; i < n; ++i) {
        if ((X && !(std::fabs(X[i]) <= 1e6)) || (V && !std::isfinite(V[i])))
            return fail(c, OIF_E_ARG, "mesh positions must be finite with |x| <= 1e6, velocities finite");
    }
    if (X) std::memcpy(&c->Xh[off], X, n * sizeof(double));
    if (V) std::memcpy(&c->Vh[off], V, n * sizeof(double));
    c->mesh_dirty = true;
    return OIF_OK;
}

int oif_read_mesh(oif_ctx* c, int oid, double* X, double* V) {
    if (!c) return OIF_E_ARG;
    if (oid != -1) {
        int rc = check_obj(c, oid);
        if (rc) return rc;
    }
    int rc = pull_mesh(c);
    if (rc) return rc;
    const size_t off = oid < 0 ? 0 : 3 * (size_t)c->obj[oid].off;
    const size_t n = oid < 0 ? 3 * (size_t)c->M : 3 * (size_t)c->obj[oid].nv;
    if (X && n) std::memcpy(X, &c->Xh[off], n * sizeof(double));
    if (V && n) std::memcpy(V, &c->Vh[off], n * sizeof(double));
    return OIF_OK;
}

int oif_step(oif_ctx* c, int n) {
    if (!c || n < 0) return OIF_E_ARG;
    if (n == 0) return OIF_OK;
    return step_impl(c, n);
}

int oif_step_timed(oif_ctx* c, int n, oif_timing* t) {
    if (!c || n <= 0 || !t) return OIF_E_ARG;
    int rc = sync_mesh(c);
    if (rc) return rc;
    HIPCALL(c, hipMemsetAsync(c->status, 0, sizeof(unsigned), c->stream));
    if ((rc = ensure_touch(c))) return rc;
    const bool split = c->overlap && !c->obj.empty();
    std::vector<StepEvents> ev((size_t)n);
    std::vector<hipEvent_t> all;
    auto mk = [&](hipEvent_t& e) -> int {
        if (hipEventCreate(&e) != hipSuccess) return OIF_E_HIP;
        all.push_back(e);
        return OIF_OK;
    };
    for (auto& E : ev) {
        if (mk(E.t0) || mk(E.t_mesh) || mk(E.t_lb)) rc = OIF_E_HIP;
        if (split && (mk(E.t_mark) || mk(E.t_wait) || mk(E.f0) || mk(E.f1))) rc = OIF_E_HIP;
    }
    for (int k = 0; k < n && !rc; ++k) {
        rc = enqueue_one(c, c->parity, c->stream, &ev[k]);
        c->parity ^= 1;
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamSynchronize(c->side);
    std::memset(t, 0, sizeof(*t));
    if (!rc) {
        auto el = [](hipEvent_t a, hipEvent_t b) {
            float v = 0;
            (void)hipEventElapsedTime(&v, a, b);
            return (double)v;
        };
        for (int k = 0; k < n; ++k) {
            const StepEvents& E = ev[k];
            if (split) {
                t->mark_ms += el(E.t0, E.t_mark);
                t->mesh_ms += el(E.t_mark, E.t_mesh);
                t->lb_ms += el(E.f0, E.f1);
                t->lb_touched_ms += el(E.t_wait, E.t_lb);
            } else {
                t->mesh_ms += el(E.t0, E.t_mesh);
                t->lb_ms += el(E.t_mesh, E.t_lb);
            }
        }
        t->total_ms = el(ev[0].t0, ev[(size_t)n - 1].t_lb);
        t->lb_ms /= n;
        t->lb_touched_ms /= n;
        t->mark_ms /= n;
        t->mesh_ms = c->obj.empty() ? 0.0 : t->mesh_ms / n;
        t->lb_launches = n;
        t->mesh_launches = c->obj.empty() ? 0 : n;
        t->overlap = split ? 1 : 0;
    }
    for (auto& e : all) (void)hipEventDestroy(e);
    if (rc) return fail(c, rc, "kernel launch failed");
    c->steps += n;
    if (c->M) c->host_stale = true;
    return watchdog(c);
}

int oif_set_graph(oif_ctx* c, int steps_per_graph) {
    if (!c || steps_per_graph < 0) return OIF_E_ARG;
    c->graph_steps = steps_per_graph > 0 ? steps_per_graph + (steps_per_graph & 1) : 0;
    drop_graph(c);
    return OIF_OK;
}

int oif_set_integrator(oif_ctx* c, int integrator) {
    if (!c) return OIF_E_ARG;
    if (integrator != OIF_INTEGRATOR_EULER && integrator != OIF_INTEGRATOR_VERLET)
        return fail(c, OIF_E_ARG, "unknown integrator");
    if (integrator == OIF_INTEGRATOR_VERLET && c->overlap)
        return fail(c, OIF_E_STATE, "overlapped stepping supports the Euler integrator only");
    int rc = pull_mesh(c);
    if (rc) return rc;
    if (integrator != c->integrator) std::fill(c->Fh.begin(), c->Fh.end(), 0.0);
    c->integrator = integrator;
    c->mesh_dirty = true;
    drop_graph(c);
    return OIF_OK;
}

int oif_read_force(oif_ctx* c, int oid, double* F) {
    if (!c || !F) return OIF_E_ARG;
    if (oid != -1) {
        int rc = check_obj(c, oid);
        if (rc) return rc;
    }
    int rc = pull_mesh(c);
    if (rc) return rc;
    const size_t off = oid < 0 ? 0 : 3 * (size_t)c->obj[oid].off;
    const size_t n = oid < 0 ? 3 * (size_t)c->M : 3 * (size_t)c->obj[oid].nv;
    if (n) std::memcpy(F, &c->Fh[off], n * sizeof(double));
    return OIF_OK;
}

int oif_write_force(oif_ctx* c, int oid, const double* F) {
    if (!c || !F) return OIF_E_ARG;
    if (c->integrator != OIF_INTEGRATOR_VERLET)
        return fail(c, OIF_E_STATE, "the carried force exists with the Verlet integrator only");
    if (oid != -1) {
        int rc = check_obj(c, oid);
        if (rc) return rc;
    }
    int rc = pull_mesh(c);
    if (rc) return rc;
    const size_t off = oid < 0 ? 0 : 3 * (size_t)c->obj[oid].off;
    const size_t n = oid < 0 ? 3 * (size_t)c->M : 3 * (size_t)c->obj[oid].nv;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(F[i])) return fail(c, OIF_E_ARG, "non-finite force");
    std::memcpy(&c->Fh[off], F, n * sizeof(double));
    c->mesh_dirty = true;
    return OIF_OK;
}

int oif_set_soft_sphere(oif_ctx* c, int type_a, int type_b, double a, double n, double cutoff, double offset) {
    if (!c) return OIF_E_ARG;
    if (type_a < 0 || type_a >= REP_TYPES || type_b < 0 || type_b >= REP_TYPES)
        return fail(c, OIF_E_ARG, "part types must lie in 0..15");
    if (!(a >= 0.0) || !std::isfinite(a) || !(n > 0.0) || !std::isfinite(n) || !(cutoff > 0.0) ||
        !std::isfinite(cutoff) || !(offset >= 0.0) || !std::isfinite(offset))
        return fail(c, OIF_E_ARG, "soft sphere: a >= 0, n > 0, cutoff > 0, offset >= 0, all finite");
    const double range = cutoff + offset;
    const int dims[3] = {c->d.nx, c->d.ny, c->d.nz};
    for (int k = 0; k < 3; ++k)
        if ((k < 2 || !c->d.walls_z) && a > 0.0 && dims[k] < 2.0 * range)
            return fail(c, OIF_E_ARG, "a periodic box length is below twice the interaction range");
    const SoftSphereDev ss{a, n, cutoff, offset};
    c->rep_pair[type_a][type_b] = ss;
    c->rep_pair[type_b][type_a] = ss;
    c->mesh_dirty = true;
    drop_graph(c);
    return OIF_OK;
}

int oif_set_wall_soft_sphere(oif_ctx* c, int type, double a, double n, double cutoff, double offset) {
    if (!c) return OIF_E_ARG;
    if (type < 0 || type >= REP_TYPES) return fail(c, OIF_E_ARG, "part types must lie in 0..15");
    if (!(a >= 0.0) || !std::isfinite(a) || !(n > 0.0) || !std::isfinite(n) || !(cutoff > 0.0) ||
        !std::isfinite(cutoff) || !(offset >= 0.0) || !std::isfinite(offset))
        return fail(c, OIF_E_ARG, "soft sphere: a >= 0, n > 0, cutoff > 0, offset >= 0, all finite");
    c->rep_wall[type] = SoftSphereDev{a, n, cutoff, offset};
    c->mesh_dirty = true;
    drop_graph(c);
    return OIF_OK;
}

int oif_set_mrt(oif_ctx* c, const double* gamma) {
    if (!c) return OIF_E_ARG;
    if (gamma)
        for (int k = 0; k < 4; ++k)
            if (!(gamma[k] > -1.0 && gamma[k] < 1.0))
                return fail(c, OIF_E_ARG, "MRT relaxation factors must lie in (-1, 1)");
    HIPCALL(c, hipStreamSynchronize(c->stream));
    c->box.mrt = gamma ? 1 : 0;
    c->box.gamma_shear = gamma ? gamma[0] : 0.0;
    c->box.gamma_bulk = gamma ? gamma[1] : 0.0;
    c->box.gamma_odd = gamma ? gamma[2] : 0.0;
    c->box.gamma_even = gamma ? gamma[3] : 0.0;
    HIPCALL(c, hipMemcpy(c->box_dev, &c->box, sizeof(BoxDev), hipMemcpyHostToDevice));
    c->mesh_dirty = true;  // batches hold copies of the box descriptor
    drop_graph(c);
    return OIF_OK;
}

int oif_set_overlap(oif_ctx* c, int on) {
    if (!c) return OIF_E_ARG;
    if (on && c->integrator == OIF_INTEGRATOR_VERLET)
        return fail(c, OIF_E_STATE, "overlapped stepping supports the Euler integrator only");
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipStreamSynchronize(c->side));
    c->overlap = on ? 1 : 0;
    c->touch_valid = false;
    drop_graph(c);
    return OIF_OK;
}

int oif_set_launch(oif_ctx* c, int lb_block, int mesh_block, int xcd_remap) {
    if (!c) return OIF_E_ARG;
    auto okb = [](int b) { return b == 64 || b == 128 || b == 256 || b == 512 || b == 1024; };
    auto okm = [](int b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
    if (lb_block >= 0 && !okb(lb_block)) return fail(c, OIF_E_ARG, "lb_block must be 64..1024, power of two");
    if (mesh_block >= 0 && !okm(mesh_block)) return fail(c, OIF_E_ARG, "mesh_block must be a multiple of 64 in 64..1024");
    if (lb_block >= 0) c->lb_block = lb_block;
    if (mesh_block >= 0) c->mesh_block = mesh_block;
    if (xcd_remap >= 0) c->remap = xcd_remap ? 1 : 0;
    drop_graph(c);
    return OIF_OK;
}

int oif_set_lb_loads(oif_ctx* c, int nontemporal) {
    if (!c) return OIF_E_ARG;
    if (nontemporal != 0 && nontemporal != 1) return fail(c, OIF_E_ARG, "nontemporal must be 0 or 1");
    c->lb_nt = nontemporal;
    drop_graph(c);
    return OIF_OK;
}

namespace {

// Who clears G.  The lattice kernel (0): one buffer serves both step parities
// (the slots a step spreads to are the ones it reads and clears, and they stay
// in cache from step to step).  The membrane kernel (1): a buffer per parity,
// so that the slots a step spread to can be zeroed while the next step
// spreads into the other one.  The switch zeroes G and the slot lists (they
// are laid out per mode).
int set_g_mode(oif_ctx* c, int by_membrane) {
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipStreamSynchronize(c->side));
    const size_t gb = g_slot(c) * (size_t)c->N;
    if (by_membrane && c->G_bytes < 2 * gb) {  // the second parity's buffer
        void* g = nullptr;
        if (hipMalloc(&g, 2 * gb) != hipSuccess) return fail(c, OIF_E_NOMEM, "hipMalloc of G failed");
        (void)hipFree(c->G);
        c->G = g;
        c->G_bytes = 2 * gb;
        c->box.G[0] = c->G;
    }
    c->box.g_by_mesh = by_membrane;
    c->box.G[1] = by_membrane ? (void*)((unsigned char*)c->G + gb) : c->G;
    HIPCALL(c, hipMemset(c->G, 0, c->G_bytes));
    HIPCALL(c, hipMemset(c->gclear, 0, 2 * sizeof(unsigned)));
    if (c->qsave_dev.p) HIPCALL(c, hipMemset(c->qsave_dev.p, 0, c->qsave_dev.n));
    HIPCALL(c, hipMemcpy(c->box_dev, &c->box, sizeof(BoxDev), hipMemcpyHostToDevice));
    return OIF_OK;
}

}  // namespace

int oif_set_force_clear(oif_ctx* c, int by_membrane) {
    if (!c) return OIF_E_ARG;
    if (by_membrane != 0 && by_membrane != 1) return fail(c, OIF_E_ARG, "by_membrane must be 0 or 1");
    if (c->box.g_by_mesh == by_membrane) return OIF_OK;
    const int rc = set_g_mode(c, by_membrane);
    if (rc) return rc;
    c->mesh_dirty = true;  // batches holding this box copy it again
    drop_graph(c);
    return OIF_OK;
}

namespace {

int read_pops(oif_ctx* c, double* out, int deviations) {
    if (!c || !out) return OIF_E_ARG;
    double* tmp = nullptr;
    const size_t n = 19 * (size_t)c->N;
    HIPCALL(c, hipMalloc(&tmp, n * 8));
    hipError_t e = launch_pops_to_f64(c->box_dev, c->N, c->d.precision, c->parity, tmp, deviations, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    HIPCALL(c, e);
    return OIF_OK;
}

int write_pops(oif_ctx* c, const double* in, int deviations) {
    if (!c || !in) return OIF_E_ARG;
    double* tmp = nullptr;
    const size_t n = 19 * (size_t)c->N;
    HIPCALL(c, hipMalloc(&tmp, n * 8));
    hipError_t e = hipMemcpyAsync(tmp, in, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_f64_to_pops(c->box_dev, c->N, c->d.precision, c->parity, tmp, deviations, c->stream);
    // both buffers: nothing streams into a solid node, which keeps its values
    if (e == hipSuccess)
        e = launch_f64_to_pops(c->box_dev, c->N, c->d.precision, c->parity ^ 1, tmp, deviations, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    HIPCALL(c, e);
    return OIF_OK;
}

}  // namespace

int oif_read_populations(oif_ctx* c, double* out) { return read_pops(c, out, 0); }
int oif_write_populations(oif_ctx* c, const double* in) { return write_pops(c, in, 0); }
int oif_read_deviations(oif_ctx* c, double* out) { return read_pops(c, out, 1); }
int oif_write_deviations(oif_ctx* c, const double* in) { return write_pops(c, in, 1); }

static int read_moments(oif_ctx* c, double* rho, double* u) {
    double* tmp = nullptr;
    const size_t n = (size_t)c->N * (rho ? 1 : 3);
    HIPCALL(c, hipMalloc(&tmp, n * 8));
    hipError_t e = launch_moments(c->box_dev, c->N, c->d.precision, c->parity, rho ? tmp : nullptr,
                                  rho ? nullptr : tmp, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rho ? rho : u, tmp, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    HIPCALL(c, e);
    return OIF_OK;
}

int oif_read_density(oif_ctx* c, double* out) {
    if (!c || !out) return OIF_E_ARG;
    return read_moments(c, out, nullptr);
}

int oif_read_velocity(oif_ctx* c, double* out) {
    if (!c || !out) return OIF_E_ARG;
    return read_moments(c, nullptr, out);
}

int oif_object_analyze(oif_ctx* c, int oid, oif_analysis* a) {
    int rc = check_obj(c, oid);
    if (rc) return rc;
    if (!a) return OIF_E_ARG;
    if ((rc = pull_mesh(c))) return rc;
    const Object& o = c->obj[oid];
    const Template& T = c->tmpl[o.tid];
    const double* X = &c->Xh[3 * (size_t)o.off];
    const double* V = &c->Vh[3 * (size_t)o.off];
    std::memset(a, 0, sizeof(*a));
    for (int k = 0; k < 3; ++k) { a->bounds[2 * k] = X[k]; a->bounds[2 * k + 1] = X[k]; }
    for (int v = 0; v < o.nv; ++v)
        for (int k = 0; k < 3; ++k) {
            a->origin[k] += X[3 * v + k];
            a->velocity[k] += V[3 * v + k];
            a->bounds[2 * k] = std::min(a->bounds[2 * k], X[3 * v + k]);
            a->bounds[2 * k + 1] = std::max(a->bounds[2 * k + 1], X[3 * v + k]);
        }
    for (int k = 0; k < 3; ++k) { a->origin[k] /= o.nv; a->velocity[k] /= o.nv; }
    double S = 0, Vol = 0;
    for (int t = 0; t < T.nt; ++t) {
        const int p = T.tri[3 * t], q = T.tri[3 * t + 1], r = T.tri[3 * t + 2];
        double n[3];
        vec_area(X, p, q, r, n);
        S += std::sqrt(vdot(n, n));
        double pa[3], pb[3], pc[3], bc[3];
        vsub(&X[3 * p], X, pa);
        vsub(&X[3 * q], X, pb);
        vsub(&X[3 * r], X, pc);
        vcross(pb, pc, bc);
        Vol -= vdot(pa, bc) / 6.0;
    }
    a->area = S;
    a->volume = Vol;
    return OIF_OK;
}

int oif_info(oif_ctx* c, oif_info_t* info) {
    if (!c || !info) return OIF_E_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_templates = (int)c->tmpl.size();
    info->n_objects = (int)c->obj.size();
    info->precision = c->d.precision;
    info->walls_z = c->d.walls_z;
    info->n_nodes = c->N;
    info->n_mesh_nodes = c->M;
    info->steps_done = c->steps;
    long long bytes = 2 * (long long)pop_bytes(c) + (long long)c->G_bytes + 8LL * ((c->N + 63) / 64);
    for (auto& b : c->tbufs) bytes += (long long)b.n;
    for (const DevBuf* b : {&c->tmpl_dev, &c->obj_dev, &c->X_dev, &c->V_dev, &c->F_dev, &c->geo_dev,
                            &c->scratch_dev, &c->qsave_dev, &c->rep_pos, &c->rep_cell, &c->rep_cnt, &c->rep_cursor,
                            &c->rep_bsum,
                            &c->rep_list, &c->rep_spos, &c->rep_stype, &c->rep_frep, &c->rep_type, &c->rep_shape})
        bytes += (long long)b->n;
    info->device_bytes = bytes;
    info->lb_block = c->lb_block;
    info->mesh_block = c->mesh_block;
    info->xcd_remap = c->remap;
    info->graph_steps = c->graph_steps;
    info->max_lds = (long long)c->max_lds;
    info->overlap = c->overlap;
    info->lds_objects = c->n_lds_obj;
    info->cpl_objects = c->n_cpl_obj;
    info->cpl_lds_bytes = (long long)c->cpl_need;
    info->force_clear_by_membrane = c->box.g_by_mesh;
    info->split_objects = c->n_split_obj;
    info->split_workgroups = c->n_split_work;
    info->split_lds_bytes = (long long)c->split_need;
    info->integrator = c->integrator;
    info->lb_nontemporal = c->lb_nt;
    return OIF_OK;
}

int oif_diagnostics(oif_ctx* c, oif_diag* d) {
    if (!c || !d) return OIF_E_ARG;
    int rc = sync_mesh(c);
    if (rc) return rc;
    double out[10];
    unsigned st = 0;
    if ((rc = run_diag(c, out, &st))) return rc;
    fill_diag(c, out, st, d);
    return OIF_OK;
}

int oif_diagnostics_noalloc(oif_ctx* c, oif_diag* d) {
    if (!c || !d) return OIF_E_ARG;
    if (c->mesh_dirty)
        return fail(c, OIF_E_STATE,
                    "oif_diagnostics_noalloc: the objects changed since the last step and their device arrays "
                    "are not in place; call oif_step (or oif_diagnostics) first");
    // partials of the lattice blocks and objects, then the totals on a
    // 256-byte boundary
    const long long nobj = (long long)c->obj.size();
    const long long max_obj = (SCRATCH_DOUBLES - 16) / 32 * 32 / 5 - c->diag_blocks;
    if (nobj > max_obj)
        return fail(c, OIF_E_ARG,
                    "oif_diagnostics_noalloc: " + std::to_string(nobj) + " objects exceed its fixed scratch (at most " +
                        std::to_string(max_obj) + ")");
    const long long fin_off = (5LL * (c->diag_blocks + nobj) + 31) / 32 * 32;
    double* part = (double*)c->scratch_addr;
    double out[10];
    unsigned st = 0;
    int rc = run_diag_in(c, part, part + fin_off, out, &st);
    if (rc) return rc;
    fill_diag(c, out, st, d);
    return OIF_OK;
}

int oif_copy_bandwidth(int device, long long bytes, int reps, double* gbps) {
    if (!gbps || bytes < 16 || reps < 1 || device < 0) return OIF_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return OIF_E_UNSUPPORTED;
    if (hipSetDevice(device) != hipSuccess) return OIF_E_HIP;
    const size_t n = (size_t)bytes & ~(size_t)15;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, n) != hipSuccess) return OIF_E_NOMEM;
    if (hipMalloc(&b, n) != hipSuccess) {
        (void)hipFree(a);
        return OIF_E_NOMEM;
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = OIF_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(a, 0, n, s) != hipSuccess ||
        launch_copy(a, b, n, s) != hipSuccess || hipEventRecord(e0, s) != hipSuccess) {
        rc = OIF_E_HIP;
    } else {
        for (int r = 0; r < reps && rc == OIF_OK; ++r)
            if (launch_copy((r & 1) ? b : a, (r & 1) ? a : b, n, s) != hipSuccess) rc = OIF_E_HIP;
        float ms = 0;
        if (rc == OIF_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = OIF_E_HIP;
        if (rc == OIF_OK) *gbps = 2.0 * (double)n * reps / (ms * 1e-3) / 1e9;
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}

int oif_touched_nodes(oif_ctx* c, long long* count) {
    if (!c || !count) return OIF_E_ARG;
    int rc = pull_mesh(c);
    if (rc) return rc;
    std::vector<unsigned char> mark((size_t)c->N, 0);
    long long cnt = 0;
    const int dims[3] = {c->d.nx, c->d.ny, c->d.nz};
    for (long long j = 0; j < c->M; ++j) {
        int i0[3];
        for (int a = 0; a < 3; ++a) i0[a] = (int)std::floor(c->Xh[3 * j + a] - 0.5);
        for (int k = 0; k < 8; ++k) {
            int ii[3];
            for (int a = 0; a < 3; ++a) {
                int v = i0[a] + ((k >> a) & 1);
                if (a == 2 && c->d.walls_z) v = std::min(std::max(v, 0), dims[2] - 1);
                v %= dims[a];
                if (v < 0) v += dims[a];
                ii[a] = v;
            }
            const size_t q = ((size_t)ii[2] * dims[1] + ii[1]) * dims[0] + ii[0];
            if (!mark[q]) { mark[q] = 1; ++cnt; }
        }
    }
    *count = cnt;
    return OIF_OK;
}

}  // extern "C"

// ===========================================================================
// autotuner: measured search of the launch shapes, cached as JSON
// ===========================================================================
namespace {

std::string tune_key(int prec, const std::vector<std::array<int, 3>>& dims, long long nobj, long long M) {
    std::ostringstream k;
    k << "gfx950|p" << prec;
    for (auto& d : dims) k << "|" << d[0] << "x" << d[1] << "x" << d[2];
    k << "|o" << nobj << "|m" << M;
    return k.str();
}

bool cache_lookup(const char* path, const std::string& key, int out[5]) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const std::string pat = "\"" + key + "\": [";
    const size_t p = s.find(pat);
    if (p == std::string::npos) return false;
    int v[5];
    if (std::sscanf(s.c_str() + p + pat.size(), "%d, %d, %d, %d, %d", &v[0], &v[1], &v[2], &v[3], &v[4]) != 5)
        return false;
    for (int k = 0; k < 5; ++k) out[k] = v[k];
    return true;
}

// Entries are [lb_block, mesh_block, xcd_remap, nontemporal, force clear by
// the membrane kernel]; entries of another form are dropped (and tuned again
// when asked for).
void cache_store(const char* path, const std::string& key, const int v[5]) {
    if (!path) return;
    std::map<std::string, std::array<int, 5>> entries;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            const size_t a = line.find('"'), b = line.find("\": [");
            if (a == std::string::npos || b == std::string::npos || b <= a) continue;
            std::array<int, 5> e{};
            if (std::sscanf(line.c_str() + b + 4, "%d, %d, %d, %d, %d", &e[0], &e[1], &e[2], &e[3], &e[4]) == 5)
                entries[line.substr(a + 1, b - a - 1)] = e;
        }
    }
    entries[key] = {v[0], v[1], v[2], v[3], v[4]};
    std::ofstream f(path);
    f << "{\n";
    size_t i = 0;
    for (auto& kv : entries) {
        f << "  \"" << kv.first << "\": [" << kv.second[0] << ", " << kv.second[1] << ", " << kv.second[2] << ", "
          << kv.second[3] << ", " << kv.second[4] << "]";
        f << (++i < entries.size() ? ",\n" : "\n");
    }
    f << "}\n";
}

// Time `n` eager steps; returns average lattice and mesh kernel times (ms).
int time_steps(oif_ctx* c, int n, double* lb_ms, double* mesh_ms) {
    oif_timing t{};
    const long long steps0 = c->steps;
    int rc = oif_step_timed(c, n, &t);
    c->steps = steps0;
    if (rc) return rc;
    *lb_ms = t.lb_ms;
    *mesh_ms = t.mesh_ms;
    return OIF_OK;
}

struct Snapshot {
    DevBuf f, x, v, F;
};

int snapshot(oif_ctx* c, Snapshot& s, bool restore) {
    const size_t pb = pop_bytes(c);
    const size_t mb = 3 * (size_t)c->M * real_size(c->d.precision);
    const size_t xb = 3 * (size_t)c->M * sizeof(double);
    if (!restore) {
        int rc;
        if ((rc = dev_alloc(c, s.f, pb))) return rc;
        if (mb && (rc = dev_alloc(c, s.x, xb))) return rc;
        if (mb && (rc = dev_alloc(c, s.v, mb))) return rc;
        if (mb && c->F_dev.p && (rc = dev_alloc(c, s.F, mb))) return rc;
        HIPCALL(c, hipMemcpyAsync(s.f.p, c->f[c->parity], pb, hipMemcpyDeviceToDevice, c->stream));
        if (mb) {
            HIPCALL(c, hipMemcpyAsync(s.x.p, c->X_dev.p, xb, hipMemcpyDeviceToDevice, c->stream));
            HIPCALL(c, hipMemcpyAsync(s.v.p, c->V_dev.p, mb, hipMemcpyDeviceToDevice, c->stream));
            if (s.F.p) HIPCALL(c, hipMemcpyAsync(s.F.p, c->F_dev.p, mb, hipMemcpyDeviceToDevice, c->stream));
        }
    } else {
        HIPCALL(c, hipMemcpyAsync(c->f[c->parity], s.f.p, pb, hipMemcpyDeviceToDevice, c->stream));
        if (mb) {
            HIPCALL(c, hipMemcpyAsync(c->X_dev.p, s.x.p, xb, hipMemcpyDeviceToDevice, c->stream));
            HIPCALL(c, hipMemcpyAsync(c->V_dev.p, s.v.p, mb, hipMemcpyDeviceToDevice, c->stream));
            if (s.F.p) HIPCALL(c, hipMemcpyAsync(c->F_dev.p, s.F.p, mb, hipMemcpyDeviceToDevice, c->stream));
        }
        HIPCALL(c, hipStreamSynchronize(c->stream));
        c->touch_valid = false;
        s.f.release();
        s.x.release();
        s.v.release();
        s.F.release();
    }
    return OIF_OK;
}

}  // namespace

extern "C" int oif_autotune(oif_ctx* c, const char* cache_path) {
    if (!c) return OIF_E_ARG;
    int rc = sync_mesh(c);
    if (rc) return rc;
    const std::string key = tune_key(c->d.precision, {{c->d.nx, c->d.ny, c->d.nz}}, (long long)c->obj.size(), c->M);
    int best[5];
    if (cache_lookup(cache_path, key, best)) {
        rc = oif_set_launch(c, best[0], best[1], best[2]);
        if (!rc) rc = oif_set_lb_loads(c, best[3]);
        return rc ? rc : oif_set_force_clear(c, best[4]);
    }
    Snapshot s;
    if ((rc = snapshot(c, s, false))) return rc;
    const int overlap = c->overlap;
    c->overlap = 0;  // time each kernel alone
    const int reps = 6;  // even: parity is unchanged after each trial
    double best_lb = 1e300, best_mesh = 1e300;
    best[0] = c->lb_block; best[1] = c->mesh_block; best[2] = c->remap; best[3] = c->lb_nt;
    best[4] = c->box.g_by_mesh;
    for (int nt : {0, 1})
        for (int lb : {128, 256, 512, 1024})
            for (int rm : {0, 1}) {
                c->lb_block = lb;
                c->remap = rm;
                c->lb_nt = nt;
                double tl, tm;
                if ((rc = time_steps(c, reps, &tl, &tm))) return rc;
                if (tl < best_lb) { best_lb = tl; best[0] = lb; best[2] = rm; best[3] = nt; }
            }
    c->lb_block = best[0];
    c->remap = best[2];
    c->lb_nt = best[3];
    if (!c->obj.empty())
        for (int mb : {128, 256, 384, 512, 640, 768, 1024}) {
            c->mesh_block = mb;
            double tl, tm;
            if ((rc = time_steps(c, reps, &tl, &tm))) return rc;
            if (tm < best_mesh) { best_mesh = tm; best[1] = mb; }
        }
    c->mesh_block = best[1];
    if (!c->obj.empty()) {
        // who clears G: the lattice kernel where it reads it, or the membrane
        // kernel from its slot lists one step later (the step time decides)
        double best_step = 1e300;
        const int g0 = c->box.g_by_mesh;
        for (int g : {0, 1}) {
            if ((rc = set_g_mode(c, g))) return rc;
            double tl, tm;
            if ((rc = time_steps(c, reps, &tl, &tm))) return rc;
            if (tl + tm < best_step) { best_step = tl + tm; best[4] = g; }
        }
        if ((rc = set_g_mode(c, best[4]))) return rc;
        if (best[4] != g0) c->mesh_dirty = true;  // batches copy the box again
    }
    c->overlap = overlap;
    if ((rc = snapshot(c, s, true))) return rc;
    c->host_stale = c->M > 0;
    drop_graph(c);
    cache_store(cache_path, key, best);
    return OIF_OK;
}

// ===========================================================================
// batching form: all boxes of a batch advance with one membrane/coupling
// launch over all objects and one lattice launch over all boxes' nodes
// ===========================================================================
namespace {

int bfail(oif_batch* b, int code, const std::string& m) {
    b->err = m;
    return code;
}

#define BHIP(b, expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return bfail(b, OIF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void bdrop_graph(oif_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->g_len = 0;
}

int batch_build(oif_batch* b) {
    for (oif_ctx* c : b->ctx) {
        int rc = sync_mesh(c);
        if (rc) return bfail(b, rc, std::string("box: ") + c->err);
    }
    bdrop_graph(b);
    // boxes and lattice work list
    // one lattice launch per kernel variant (obstacles or not, MRT or BGK),
    // so that every box runs the kernel it runs on its own
    std::vector<BoxDev> boxes;
    std::vector<int2> work;
    for (size_t i = 0; i < b->ctx.size(); ++i) boxes.push_back(b->ctx[i]->box);
    for (int v = 0; v < 4; ++v) {
        b->var_off[v] = (int)work.size();
        for (size_t i = 0; i < b->ctx.size(); ++i) {
            const oif_ctx* c = b->ctx[i];
            if ((c->n_bnd > 0 ? 1 : 0) + 2 * c->box.mrt != v) continue;
            const int nb = (c->N + b->lb_block - 1) / b->lb_block;
            for (int k = 0; k < nb; ++k) work.push_back(make_int2((int)i, k));
        }
    }
    b->var_off[4] = (int)work.size();
    b->nblocks = (int)work.size();
    b->boxes_dev.release();
    b->work_dev.release();
    BHIP(b, hipMalloc(&b->boxes_dev.p, boxes.size() * sizeof(BoxDev)));
    BHIP(b, hipMalloc(&b->work_dev.p, work.size() * sizeof(int2)));
    BHIP(b, hipMemcpy(b->boxes_dev.p, boxes.data(), boxes.size() * sizeof(BoxDev), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->work_dev.p, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice));
    // objects of all boxes: LDS-resident group first, each largest mesh first
    const size_t osz = objdev_size(b->precision);
    struct Ent { const unsigned char* p; int group; int nv; size_t need, cpl, split; int box; int nslice; };
    std::vector<Ent> ents;
    for (size_t bi = 0; bi < b->ctx.size(); ++bi) {
        oif_ctx* c = b->ctx[bi];
        const size_t n = c->obj.size();
        for (size_t k = 0; k < n; ++k) {
            const unsigned char* p = c->obj_host.data() + k * osz;
            const int kk = (int)k;
            const int group = kk < c->n_lds_obj ? 0
                              : kk < c->n_lds_obj + c->n_split_obj ? 1
                              : kk < c->n_lds_obj + c->n_split_obj + c->n_cpl_obj ? 2 : 3;
            // the template pointer of the sorted entry says which mesh it is
            const void* tptr = b->precision == OIF_PREC_FP64 ? (const void*)((const ObjDev<double>*)p)->t
                                                            : (const void*)((const ObjDev<float>*)p)->t;
            const size_t tsz = b->precision == OIF_PREC_FP64 ? sizeof(TmplDev<double>) : sizeof(TmplDev<float>);
            const size_t tid = ((const unsigned char*)tptr - (const unsigned char*)c->tmpl_dev.p) / tsz;
            const Template& T = c->tmpl[tid];
            ents.push_back({p, group, T.nv,
                            mesh_lds_bytes(b->precision, T.nv, T.nt, T.ne, T.ucap, T.ccap, tmpl_conservative(T)),
                            mesh_cpl_lds_bytes(b->precision, T.nv, T.nt, T.ne, T.ucap, T.ccap,
                                               tmpl_conservative(T)),
                            split_need_bytes(b->precision, T),
                            (int)bi, T.nslice});
        }
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& c) {
        if (a.group != c.group) return a.group < c.group;
        return a.nv > c.nv;
    });
    std::vector<unsigned char> host(ents.size() * osz);
    b->n_lds_obj = 0;
    b->n_split_obj = 0;
    b->n_cpl_obj = 0;
    b->lds_need = 0;
    b->split_need = 0;
    b->cpl_need = 0;
    b->p_cpl_need = 0;
    b->any_conservative = 0;
    b->any_lists = 0;
    for (oif_ctx* c : b->ctx) b->any_lists |= c->box.g_by_mesh;
    std::vector<int2> sw;  // split launches' workgroups
    for (oif_ctx* c : b->ctx)
        for (const Template& T : c->tmpl) b->any_conservative |= tmpl_conservative(T);
    for (size_t k = 0; k < ents.size(); ++k) {
        std::memcpy(host.data() + k * osz, ents[k].p, osz);
        if (ents[k].group == 0) {
            ++b->n_lds_obj;
            b->lds_need = std::max(b->lds_need, ents[k].need);
        } else if (ents[k].group == 1) {
            for (int sl = 0; sl < ents[k].nslice; ++sl) sw.push_back(make_int2(b->n_split_obj, sl));
            ++b->n_split_obj;
            b->split_need = std::max(b->split_need, ents[k].split);
            b->p_cpl_need = std::max(b->p_cpl_need, ents[k].cpl);
        } else if (ents[k].group == 2) {
            ++b->n_cpl_obj;
            b->cpl_need = std::max(b->cpl_need, ents[k].cpl);
            b->p_cpl_need = std::max(b->p_cpl_need, ents[k].cpl);
        }
    }
    b->n_split_work = (int)sw.size();
    b->split_work.release();
    if (!sw.empty()) {
        BHIP(b, hipMalloc(&b->split_work.p, sw.size() * sizeof(int2)));
        BHIP(b, hipMemcpy(b->split_work.p, sw.data(), sw.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    b->nobj = (int)ents.size();
    b->obj_dev.release();
    BHIP(b, hipMalloc(&b->obj_dev.p, host.size() + 16));
    if (!host.empty()) BHIP(b, hipMemcpy(b->obj_dev.p, host.data(), host.size(), hipMemcpyHostToDevice));
    if (b->persistent) {
        // Task list of the persistent form: membrane tasks largest mesh first
        // (the longest chains start first), then the lattice blocks of the
        // boxes in the order their membranes should finish (smallest largest
        // mesh first, then fewest objects).
        for (oif_ctx* c : b->ctx)
            if (c->n_bnd > 0 || c->box.mrt)
                return bfail(b, OIF_E_UNSUPPORTED,
                             "the persistent batch form runs boxes without obstacles with the BGK collision only");
        std::vector<int> mo(ents.size());
        for (size_t k = 0; k < mo.size(); ++k) mo[k] = (int)k;
        std::stable_sort(mo.begin(), mo.end(), [&](int a, int c) { return ents[a].nv > ents[c].nv; });
        std::vector<unsigned char> pobj(ents.size() * osz), pgroup(ents.size() + 1, 0);
        std::vector<int> pbox(ents.size() + 1, 0), bn(b->ctx.size(), 0), bmax(b->ctx.size(), 0);
        for (size_t k = 0; k < mo.size(); ++k) {
            const Ent& e = ents[mo[k]];
            std::memcpy(pobj.data() + k * osz, e.p, osz);
            // the persistent kernel runs split objects whole, with the coupling
            // area in LDS
            pgroup[k] = (unsigned char)(e.group == 0 ? 0 : (e.group <= 2 ? 1 : 2));
            pbox[k] = e.box;
            ++bn[e.box];
            bmax[e.box] = std::max(bmax[e.box], e.nv);
        }
        std::vector<int> bo(b->ctx.size());
        for (size_t i = 0; i < bo.size(); ++i) bo[i] = (int)i;
        std::stable_sort(bo.begin(), bo.end(), [&](int a, int c) {
            return bmax[a] != bmax[c] ? bmax[a] < bmax[c] : bn[a] < bn[c];
        });
        const int block = b->mesh_block;
        b->p_lds = std::max(b->n_lds_obj ? b->lds_need : 0, b->p_cpl_need);
        int per_cu = 0, dev = 0, ncu = 0;
        BHIP(b, hipGetDevice(&dev));
        BHIP(b, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        BHIP(b, batch_blocks_per_cu(b->precision, b->lb_nt, block, b->p_lds, &per_cu));
        if (per_cu < 1) return bfail(b, OIF_E_UNSUPPORTED, "persistent batch: no workgroup fits a compute unit");
        const int slots = per_cu * ncu;
        long long nblk_all = 0;
        for (oif_ctx* c : b->ctx) nblk_all += (c->N + block - 1) / block;
        // lattice blocks per task: by default about three lattice tasks per
        // resident workgroup (fewer tickets and waits; enough tasks to even
        // out the ends of the boxes' membrane phases)
        b->p_chunk = b->p_chunk_req > 0
                         ? b->p_chunk_req
                         : (int)std::max(1LL, std::min(64LL, (nblk_all + 3LL * slots - 1) / (3LL * slots)));
        std::vector<int2> lbw;
        for (int i : bo) {
            const int nb = (b->ctx[i]->N + block - 1) / block;
            for (int k = 0; k < nb; k += b->p_chunk) lbw.push_back(make_int2(i, k));
        }
        const int ntasks = (int)(ents.size() + lbw.size());
        b->p_grid = std::max(1, std::min(slots, ntasks));
        const size_t nctr = 2 * (3 + b->ctx.size());
        for (DevBuf* d : {&b->sched_dev, &b->p_objs, &b->p_group, &b->p_objbox, &b->p_lbwork, &b->p_boxnmesh, &b->p_ctr})
            d->release();
        BHIP(b, hipMalloc(&b->p_objs.p, pobj.size() + 16));
        BHIP(b, hipMalloc(&b->p_group.p, pgroup.size()));
        BHIP(b, hipMalloc(&b->p_objbox.p, pbox.size() * sizeof(int)));
        BHIP(b, hipMalloc(&b->p_lbwork.p, (lbw.size() + 1) * sizeof(int2)));
        BHIP(b, hipMalloc(&b->p_boxnmesh.p, bn.size() * sizeof(int)));
        BHIP(b, hipMalloc(&b->p_ctr.p, nctr * sizeof(unsigned)));
        BHIP(b, hipMalloc(&b->sched_dev.p, sizeof(BatchSched)));
        if (!pobj.empty()) BHIP(b, hipMemcpy(b->p_objs.p, pobj.data(), pobj.size(), hipMemcpyHostToDevice));
        BHIP(b, hipMemcpy(b->p_group.p, pgroup.data(), pgroup.size(), hipMemcpyHostToDevice));
        BHIP(b, hipMemcpy(b->p_objbox.p, pbox.data(), pbox.size() * sizeof(int), hipMemcpyHostToDevice));
        if (!lbw.empty()) BHIP(b, hipMemcpy(b->p_lbwork.p, lbw.data(), lbw.size() * sizeof(int2), hipMemcpyHostToDevice));
        BHIP(b, hipMemcpy(b->p_boxnmesh.p, bn.data(), bn.size() * sizeof(int), hipMemcpyHostToDevice));
        BHIP(b, hipMemset(b->p_ctr.p, 0, nctr * sizeof(unsigned)));
        BatchSched& S = b->sched;
        S.ntasks = ntasks;
        S.nmesh = (int)ents.size();
        S.nbox = (int)b->ctx.size();
        S.objs = b->p_objs.p;
        S.group = (const unsigned char*)b->p_group.p;
        S.obj_box = (const int*)b->p_objbox.p;
        S.lbwork = (const int2*)b->p_lbwork.p;
        S.lb_chunk = b->p_chunk;
        S.boxes = (const BoxDev*)b->boxes_dev.p;
        S.box_nmesh = (const int*)b->p_boxnmesh.p;
        S.ctr = (unsigned*)b->p_ctr.p;
        S.spin_limit = 1ull << 16;  // ~0.1 s of polling; a box's membranes take well under 1 ms
        BHIP(b, hipMemcpy(b->sched_dev.p, &S, sizeof(BatchSched), hipMemcpyHostToDevice));
    }
    b->built = true;
    return OIF_OK;
}

int batch_enqueue(oif_batch* b, int n, int parity0, hipStream_t s, std::vector<hipEvent_t>* ev) {
    int par = parity0;
    const size_t osz = objdev_size(b->precision);
    for (int k = 0; k < n; ++k) {
        if (ev) (void)hipEventRecord((*ev)[3 * k], s);
        for (oif_ctx* c : b->ctx)
            if (c->rep_on)
                BHIP(b, launch_repulsion(c->rep_h, (const RepDev*)c->rep_desc.p, c->obj_dev.p,
                                         (int)c->obj.size(), c->d.precision, s));
        if (b->persistent) {  // the membranes and the lattice of every box in one launch
            BatchLaunch bl{(const BatchSched*)b->sched_dev.p, b->p_grid, b->mesh_block, b->p_lds, par,
                           b->precision, b->lb_nt, s};
            BHIP(b, launch_batch(bl));
            if (ev) {
                (void)hipEventRecord((*ev)[3 * k + 1], s);
                (void)hipEventRecord((*ev)[3 * k + 2], s);
            }
            par ^= 1;
            continue;
        }
        MeshLaunch ml{};
        ml.block = b->mesh_block;
        ml.parity = par;
        ml.precision = b->precision;
        ml.conservative = b->any_conservative;
        ml.stream = s;
        ml.lists = b->any_lists;
        if (b->n_lds_obj > 0) {
            ml.objs = b->obj_dev.p;
            ml.nobj = b->n_lds_obj;
            ml.lds_bytes = b->lds_need;
            BHIP(b, launch_mesh(ml));
        }
        if (b->n_split_obj > 0) {
            MeshLaunch sl = ml;
            sl.objs = (const unsigned char*)b->obj_dev.p + osz * b->n_lds_obj;
            sl.nobj = b->n_split_obj;
            sl.lds_bytes = 0;
            sl.work = (const int2*)b->split_work.p;
            sl.nwork = b->n_split_work;
            sl.split_lds = b->split_need;
            BHIP(b, launch_mesh(sl));
        }
        if (b->n_cpl_obj > 0) {
            ml.objs = (const unsigned char*)b->obj_dev.p + osz * (b->n_lds_obj + b->n_split_obj);
            ml.nobj = b->n_cpl_obj;
            ml.lds_bytes = 0;
            ml.cpl_lds_bytes = b->cpl_need;
            BHIP(b, launch_mesh(ml));
        }
        const int done = b->n_lds_obj + b->n_split_obj + b->n_cpl_obj;
        if (b->nobj > done) {
            ml.objs = (const unsigned char*)b->obj_dev.p + osz * done;
            ml.nobj = b->nobj - done;
            ml.lds_bytes = 0;
            ml.cpl_lds_bytes = 0;
            BHIP(b, launch_mesh(ml));
        }
        if (ev) (void)hipEventRecord((*ev)[3 * k + 1], s);
        for (int v = 0; v < 4; ++v) {
            LbLaunch ll{(const BoxDev*)b->boxes_dev.p, (const int2*)b->work_dev.p + b->var_off[v],
                        b->var_off[v + 1] - b->var_off[v], b->lb_block, par, b->remap, b->precision, s,
                        LB_ALL, v & 1, v >> 1, b->lb_nt};
            if (ll.nblocks > 0) BHIP(b, launch_lb(ll));
        }
        if (ev) (void)hipEventRecord((*ev)[3 * k + 2], s);
        par ^= 1;
    }
    return OIF_OK;
}

int batch_prepare(oif_batch* b) {
    bool dirty = !b->built;
    for (oif_ctx* c : b->ctx) dirty = dirty || c->mesh_dirty;
    const int par = b->ctx[0]->parity;
    for (oif_ctx* c : b->ctx)
        if (c->parity != par) return bfail(b, OIF_E_STATE, "boxes of a batch must be at the same step parity");
    if (dirty) return batch_build(b);
    return OIF_OK;
}

int batch_finish(oif_batch* b, int n) {
    if (b->persistent && b->p_ctr.p) {
        // the wait-limit flags of both step parities
        const size_t per = 3 + b->ctx.size();
        unsigned f[2] = {0, 0};
        hipStream_t s = b->ctx[0]->stream;
        BHIP(b, hipMemcpyAsync(&f[0], (unsigned*)b->p_ctr.p + 2, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        BHIP(b, hipMemcpyAsync(&f[1], (unsigned*)b->p_ctr.p + per + 2, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        BHIP(b, hipStreamSynchronize(s));
        if (f[0] | f[1]) {
            BHIP(b, hipMemset(b->p_ctr.p, 0, 2 * per * sizeof(unsigned)));
            return bfail(b, OIF_E_HIP, "persistent batch: a lattice task waited past its limit for the membranes "
                                       "of its box; the step's results are not valid");
        }
    }
    for (oif_ctx* c : b->ctx) {
        c->parity ^= (n & 1);
        c->steps += n;
        c->touch_valid = false;  // batched steps do not mark stencils
        if (c->M) c->host_stale = true;
    }
    for (oif_ctx* c : b->ctx) {
        int rc = watchdog(c);
        if (rc) return bfail(b, rc, c->err);
    }
    return OIF_OK;
}

}  // namespace

extern "C" {

int oif_batch_create(oif_ctx* const* boxes, int n, oif_batch** out) {
    if (!boxes || n <= 0 || !out) return OIF_E_ARG;
    *out = nullptr;
    for (int i = 0; i < n; ++i)
        if (!boxes[i] || boxes[i]->d.precision != boxes[0]->d.precision || boxes[i]->d.device != boxes[0]->d.device)
            return OIF_E_ARG;
    std::unique_ptr<oif_batch> b(new oif_batch());
    b->ctx.assign(boxes, boxes + n);
    b->precision = boxes[0]->d.precision;
    b->lb_block = boxes[0]->lb_block;
    b->mesh_block = boxes[0]->mesh_block;
    b->remap = boxes[0]->remap;
    b->lb_nt = boxes[0]->lb_nt;
    *out = b.release();
    return OIF_OK;
}

int oif_batch_destroy(oif_batch* b) {
    if (!b) return OIF_OK;
    if (!b->ctx.empty()) (void)hipStreamSynchronize(b->ctx[0]->stream);
    bdrop_graph(b);
    b->boxes_dev.release();
    b->work_dev.release();
    b->obj_dev.release();
    b->split_work.release();
    for (DevBuf* d : {&b->sched_dev, &b->p_objs, &b->p_group, &b->p_objbox, &b->p_lbwork, &b->p_boxnmesh, &b->p_ctr})
        d->release();
    delete b;
    return OIF_OK;
}

const char* oif_batch_last_error(const oif_batch* b) { return b ? b->err.c_str() : "null batch"; }

int oif_batch_set_graph(oif_batch* b, int steps_per_graph) {
    if (!b || steps_per_graph < 0) return OIF_E_ARG;
    b->graph_steps = steps_per_graph > 0 ? steps_per_graph + (steps_per_graph & 1) : 0;
    bdrop_graph(b);
    return OIF_OK;
}

int oif_batch_set_launch(oif_batch* b, int lb_block, int mesh_block, int xcd_remap) {
    if (!b) return OIF_E_ARG;
    auto okb = [](int v) { return v == 64 || v == 128 || v == 256 || v == 512 || v == 1024; };
    auto okm = [](int v) { return v >= 64 && v <= 1024 && v % 64 == 0; };
    if ((lb_block >= 0 && !okb(lb_block)) || (mesh_block >= 0 && !okm(mesh_block))) return OIF_E_ARG;
    if (lb_block >= 0) b->lb_block = lb_block;
    if (mesh_block >= 0) b->mesh_block = mesh_block;
    if (xcd_remap >= 0) b->remap = xcd_remap ? 1 : 0;
    b->built = false;
    bdrop_graph(b);
    return OIF_OK;
}

int oif_batch_set_persistent(oif_batch* b, int on, int lattice_blocks_per_task) {
    if (!b || (on != 0 && on != 1) || lattice_blocks_per_task < 0) return OIF_E_ARG;
    b->persistent = on;
    b->p_chunk_req = lattice_blocks_per_task;
    b->built = false;
    bdrop_graph(b);
    return OIF_OK;
}

int oif_batch_set_lb_loads(oif_batch* b, int nontemporal) {
    if (!b || (nontemporal != 0 && nontemporal != 1)) return OIF_E_ARG;
    b->lb_nt = nontemporal;
    bdrop_graph(b);
    return OIF_OK;
}

int oif_batch_step(oif_batch* b, int n) {
    if (!b || n < 0) return OIF_E_ARG;
    if (n == 0) return OIF_OK;
    int rc = batch_prepare(b);
    if (rc) return rc;
    hipStream_t s = b->ctx[0]->stream;
    for (oif_ctx* c : b->ctx) BHIP(b, hipMemsetAsync(c->status, 0, sizeof(unsigned), s));
    int par = b->ctx[0]->parity;
    int left = n;
    if (b->graph_steps > 0 && n >= b->graph_steps) {
        if (par) {
            if ((rc = batch_enqueue(b, 1, par, s, nullptr))) return rc;
            par ^= 1;
            --left;
        }
        if (!b->gexec || b->g_len != b->graph_steps) {
            bdrop_graph(b);
            hipGraph_t g = nullptr;
            BHIP(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            rc = batch_enqueue(b, b->graph_steps, 0, s, nullptr);
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
            BHIP(b, e2);
            hipError_t e3 = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            BHIP(b, e3);
            b->g_len = b->graph_steps;
        }
        while (left >= b->graph_steps) {
            BHIP(b, hipGraphLaunch(b->gexec, s));
            left -= b->graph_steps;
        }
    }
    if (left > 0 && (rc = batch_enqueue(b, left, par, s, nullptr))) return rc;
    return batch_finish(b, n);
}

int oif_batch_step_timed(oif_batch* b, int n, oif_timing* t) {
    if (!b || n <= 0 || !t) return OIF_E_ARG;
    int rc = batch_prepare(b);
    if (rc) return rc;
    hipStream_t s = b->ctx[0]->stream;
    for (oif_ctx* c : b->ctx) BHIP(b, hipMemsetAsync(c->status, 0, sizeof(unsigned), s));
    std::vector<hipEvent_t> ev(3 * (size_t)n);
    for (auto& e : ev) BHIP(b, hipEventCreate(&e));
    rc = batch_enqueue(b, n, b->ctx[0]->parity, s, &ev);
    (void)hipStreamSynchronize(s);
    double lb = 0, ms = 0;
    float v = 0;
    for (int k = 0; k < n && !rc; ++k) {
        (void)hipEventElapsedTime(&v, ev[3 * k], ev[3 * k + 1]);
        ms += v;
        (void)hipEventElapsedTime(&v, ev[3 * k + 1], ev[3 * k + 2]);
        lb += v;
    }
    (void)hipEventElapsedTime(&v, ev[0], ev[3 * (size_t)n - 1]);
    t->total_ms = v;
    t->lb_ms = lb / n;
    t->mesh_ms = ms / n;
    t->lb_launches = n;
    t->mesh_launches = n;
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    return batch_finish(b, n);
}

int oif_batch_autotune(oif_batch* b, const char* cache_path) {
    if (!b) return OIF_E_ARG;
    std::vector<std::array<int, 3>> dims;
    long long nobj = 0, M = 0;
    for (oif_ctx* c : b->ctx) {
        dims.push_back({c->d.nx, c->d.ny, c->d.nz});
        nobj += (long long)c->obj.size();
        M += c->M;
    }
    const std::string key = tune_key(b->precision, dims, nobj, M);
    int best[5] = {b->lb_block, b->mesh_block, b->remap, b->lb_nt, 0};
    if (cache_lookup(cache_path, key, best)) {
        const int rc = oif_batch_set_launch(b, best[0], best[1], best[2]);
        return rc ? rc : oif_batch_set_lb_loads(b, best[3]);
    }
    int rc = batch_prepare(b);
    if (rc) return rc;
    std::vector<Snapshot> snaps(b->ctx.size());
    for (size_t i = 0; i < b->ctx.size(); ++i)
        if ((rc = snapshot(b->ctx[i], snaps[i], false))) return bfail(b, rc, b->ctx[i]->err);
    const int reps = 6;
    double best_lb = 1e300, best_mesh = 1e300;
    auto trial = [&](double* tl, double* tm) -> int {
        oif_timing t{};
        std::vector<long long> st;
        for (oif_ctx* c : b->ctx) st.push_back(c->steps);
        int r = oif_batch_step_timed(b, reps, &t);
        for (size_t i = 0; i < b->ctx.size(); ++i) b->ctx[i]->steps = st[i];
        *tl = t.lb_ms;
        *tm = t.mesh_ms;
        return r;
    };
    for (int nt : {0, 1})
        for (int lb : {128, 256, 512, 1024})
            for (int rm : {0, 1}) {
                oif_batch_set_launch(b, lb, -1, rm);
                oif_batch_set_lb_loads(b, nt);
                double tl, tm;
                if ((rc = trial(&tl, &tm))) return rc;
                if (tl < best_lb) { best_lb = tl; best[0] = lb; best[2] = rm; best[3] = nt; }
            }
    oif_batch_set_launch(b, best[0], -1, best[2]);
    oif_batch_set_lb_loads(b, best[3]);
    for (int mb : {128, 256, 384, 512, 640, 768, 1024}) {
        oif_batch_set_launch(b, -1, mb, -1);
        double tl, tm;
        if ((rc = trial(&tl, &tm))) return rc;
        if (tm < best_mesh) { best_mesh = tm; best[1] = mb; }
    }
    oif_batch_set_launch(b, best[0], best[1], best[2]);
    for (size_t i = 0; i < b->ctx.size(); ++i)
        if ((rc = snapshot(b->ctx[i], snaps[i], true))) return bfail(b, rc, b->ctx[i]->err);
    cache_store(cache_path, key, best);
    return OIF_OK;
}

}  // extern "C"
