// oif_device.h -- device-side data layout of the coupled LB / membrane step
// and the launchers the host runtime calls.  Internal to liboif.so.
//
// HBM layout of one box (context):
//   f[2]   two population buffers of the storage type, holding deviations
//          n_i - w_i rho0, nodes numbered x fastest, then y, then z; tiles of
//          64 consecutive nodes, each tile [19][64] (value (i, p) at element
//          ((p / 64) * 19 + i) * 64 + p % 64, N rounded up to whole tiles);
//          the step reads f[parity] and writes f[parity ^ 1]
//   G[2]   coupling force density per step parity (a step of parity k spreads
//          into G[k]), [N][4] (x, y, z, unused: one 32-byte slot per node):
//          double (FP64 form) or int64 fixed point with resolution 2^-e (FP32
//          forms, order-independent sums).  The lattice kernel only reads it:
//          each membrane workgroup keeps the list of slots it added to and
//          zeroes them in the next step, when the lattice kernel is done with
//          them (gclear covers a workgroup that spread corner by corner)
//   mask   one bit per node, set where G is non-zero; the lattice kernel reads
//          G only where a bit is set and clears the bit
//   X, V   mesh node positions (absolute, unwrapped, FP64 in every form, so
//          that edge lengths and areas near their relaxed values do not lose
//          their digits to position round-off; an integer per-object anchor is
//          added to the stencil index and is 0 here) and velocities ([M][3],
//          compute type)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oif {

enum : int { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16 = 2, PREC_BF16 = 3 };
enum : unsigned { ST_NONFINITE = 1u, ST_CLAMPED = 2u, ST_OVERFLOW = 4u };

struct BoxDev {
    int nx, ny, nz, walls_z;
    int N;
    int precision;
    // node index -> coordinates without a hardware divide: for d = nx or ny,
    // q / d = umulhi(q, div) >> sh for every q < 2^31 (div = 0 marks d = 1)
    unsigned div_nx, div_ny;
    int sh_nx, sh_ny;
    void* f[2];
    void* G[2];
    // [2] per step parity, used when the membrane kernel clears G: set when a
    // workgroup of that step spread without a list of its slots (corner by
    // corner); the lattice kernel then clears G[parity] where it reads it.
    // Reset by the membrane launch of the next step.
    unsigned* gclear;
    // 1: the membrane workgroups keep lists of the slots they add to and zero
    // them one step later (G[0] and G[1] distinct); 0: they keep none and the
    // lattice kernel clears G where it reads it (G[0] == G[1])
    int g_by_mesh;
    unsigned long long* mask;
    // Split (overlapped) stepping, double-buffered by population parity:
    // touch[k] has one bit per node inside some mesh node's 2x2x2 stencil at
    // the start of a step of parity k.
    unsigned long long* touch[2];
    // Obstacles (null when the box has none): boundary id per node (0 = fluid);
    // per node a link word: bit 0 = the node is solid, bit i (1..18) = the push
    // in direction i ends in a solid node, bits 23..30 = the id of the moving
    // boundary when all of the node's solid neighbours belong to it, bit 31 =
    // solid neighbours of several boundaries, one of them moving (look each
    // up); the wall velocity of each boundary id ([256][3]).
    const unsigned char* btype;
    const unsigned* links;
    const double* wall_u;
    unsigned* status;
    double g[3];
    double rho0;
    double omega;   // 1 / tau
    double guo;     // 1 - 1/(2 tau)
    double xi;
    float st_scale; // storage scale of deviations (2^s for FP16, else 1)
    float st_inv;
    double fp_scale; // fixed-point scale 2^e
    double fp_inv;
    // collision: 0 = BGK (omega, guo); 1 = multiple relaxation times with the
    // factors of the shear and bulk stress and of the odd and even
    // non-hydrodynamic parts
    int mrt;
    double gamma_shear, gamma_bulk, gamma_odd, gamma_even;
};

template <typename real>
struct TmplDev {
    int nv, nt, ne;
    int linear;
    const int* tri;        // [nt][3]
    // Per-node incidence lists (CSR).  Each entry holds everything the node's
    // gather needs besides LDS data, so the entries of a node are independent
    // loads with no second indirection.
    const int4* n_off;     // [nv + 1] (edge, hinge, triangle) list offsets
    const int2* e_inc;     // (neighbour node, edge id)
    const int4* h_inc;     // (hinge id << 2 | role, T1, T2, 0); role 0 = A, 1 = B, 2 = C, 3 = D
    const int4* t_inc;     // (triangle, next vertex, vertex after that, 0) in the triangle's order
    const double* L0;      // [ne] (FP64: L - L0 cancels near the relaxed shape)
    const int4* hinge;     // (A, B, C, D): T1 = (A, B, C) runs B -> C, T2 has wing D
    const double* theta0;  // [ne] relaxed inner dihedral angle
    const double2* cs0;    // [ne] cos and sin of theta0 - pi (FP64)
    const double* S0;      // [nt] (FP64: S - S0 cancels near the relaxed shape)
    const double* hbar;    // [ne] mean relaxed wing height (conservative model)
    int conservative;      // force model: 0 = the paper's rules, 1 = conservative
    double Sg0, V0;
    double ks, kb, kal, kag, kv;
    int ucap;              // lattice nodes of the largest stencil box kept in LDS
    int ccap;              // touched lattice nodes an object may have in LDS
    // Split launches (meshes too large for LDS): nslice workgroups per object;
    // slice k updates the nodes order[slice_off[k] .. slice_off[k + 1]), a
    // compact patch of the reference shape, of at most smax nodes, through its
    // sub-template subs[k]: the patch's nodes (numbered 0 .. slice_off[1] - 1
    // there) and the other nodes its triangles and hinges reach, those
    // triangles and hinges, and the incidence lists of the patch's nodes, all
    // in local numbering; its order maps local node numbers to the object's.
    // A sub-template keeps the template's nslice, smax, capacities and moduli.
    int nslice, smax;
    const int* order;      // [nv]
    const int* slice_off;  // [nslice + 1]
    const TmplDev* subs;   // [nslice], null when nslice == 1
};

// Per-object LDS (or global scratch) layout of the membrane kernel, R = the
// arithmetic type:
//   fs  elastic force per node, R [nv][3]
//   then a region used twice:
//     forces phase:  xs  node positions, FP64 [nv][3]
//                    tn  unit inward normal + area per triangle, R [nt][4]
//                    tr  (S - S0)/S per triangle, R [nt]
//                    se  stretching coefficient per edge, R [ne]
//                    fh  bending coefficients per edge: R [ne] (the paper's
//                        magnitude) or R [ne][4] (conservative model: wing
//                        factors c/h_A, c/h_D and foot positions a_A, a_D)
//     coupling phase: need  one bit per node of the object's stencil box
//                     pre   exclusive popcount prefix per bit word
//                     ug    fluid velocity at the touched nodes, R [ccap][3]
//                     qn    their lattice indices, int [ccap]
//                     gacc  summed reaction force, 8-byte accumulators [ccap][3]
// (the coupling phase reads the node positions from HBM again, so the
// positions need not outlive the forces phase)
struct MeshLayout {
    size_t fs, xs, tn, tr, se, fh, need, nwords, ug, qn, gacc, total;
};
__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }
__host__ __device__ inline MeshLayout mesh_layout(size_t r, int nv, int nt, int ne, int ucap, int ccap,
                                                   int cons) {
    MeshLayout L;
    L.fs = 0;
    L.xs = align16((size_t)nv * 3 * r);
    L.tn = align16(L.xs + (size_t)nv * 3 * sizeof(double));
    L.tr = L.tn + (size_t)nt * 4 * r;
    L.se = align16(L.tr + (size_t)nt * r);
    L.fh = align16(L.se + (size_t)ne * r);
    const size_t end_forces = L.fh + (size_t)ne * r * (cons ? 4 : 1);
    L.need = L.xs;
    L.nwords = ((size_t)ucap + 31) / 32;
    L.ug = align16(L.need + 2 * L.nwords * 4);
    L.qn = L.ug + (size_t)ccap * 3 * r;
    L.gacc = align16(L.qn + (size_t)ccap * 4);
    // summed reaction force: 3 int64 words per node (FP32 forms), 6 (FP64)
    const size_t end_coupling = L.gacc + (size_t)ccap * (r == 8 ? 6 : 3) * 8;
    L.total = align16(end_forces > end_coupling ? end_forces : end_coupling);
    return L;
}

// Split launches (meshes too large for LDS whose positions fit there): the
// phase a membrane launch runs (all of it, or one of the two split launches)
enum { PH_ALL = 0, PH_SUMS = 1, PH_PATCH = 2 };
// LDS of the split launches: the sums launch holds the object's positions
// (FP64 [nv][3]); the patch launch the mesh layout of the patch's
// sub-template.  The object's scratch: its mesh layout, then the area and
// volume sums of each slice (double [nslice][2]).
__host__ __device__ inline size_t split_part_offset(const MeshLayout& L) { return align16(L.total); }

template <typename real>
struct ObjDev {
    const TmplDev<real>* t;
    const BoxDev* box;
    double* X;        // [nv][3] object-local positions (FP64 in every form)
    real* V;          // [nv][3]
    double* geo;      // [2]: total area, volume at the start of the last step
    // velocity Verlet (null: symplectic Euler): the total force of the last
    // step, [nv][3], carried into the first half kick of the next
    real* F;
    // soft-sphere repulsion (null: none): this step's force on each node,
    // [nv][3], computed before the membrane kernel and added to the total
    const real* frep;
    int node0;        // index of the object's first node among all mesh nodes
    int anchor[3];
    real inv_mass;
    real fext[3];
    double mass;
    unsigned char* scratch; // global stand-in for LDS when the mesh does not fit
    // slots of G this object's workgroups added to, per step parity and slice:
    // [2][nslice][1 + ccap] ints (a count, then lattice node indices)
    int* qsave;
};

// ---- soft-sphere repulsion ---------------------------------------------------
// a (d - offset)^-n for offset < d < offset + cutoff; a == 0: no interaction
struct SoftSphereDev {
    double a, n, cutoff, offset;
};
// Obstacle shape for the wall repulsion.  kind 0: rhomboid corner + s a + t b
// + u c (s, t, u in [0, 1]); kind 1: half-space n.x < dist (n unit).
struct ShapeDev {
    int kind;
    double corner[3], e[3][3];  // rhomboid corner and edge vectors a, b, c
    double cof[3][3], det;      // b x c, c x a, a x b and a . (b x c)
    double n[3], dist;          // half-space
};
constexpr int REP_TYPES = 16;   // part types 0 .. 15
// Cell lists of one box: the mesh nodes sorted by cell (cells of at least the
// largest pair range, a regular grid over the box, x fastest), inside a cell
// by node id; positions and types copied into that order, so that a node's
// partners are read from contiguous runs.
struct RepDev {
    int M;
    int ncell;
    int nc[3];
    double hc[3];               // cell edge per axis (>= the pair range)
    double L[3];
    double range2;              // square of the largest pair range
    int walls_z, pairs;         // pairs: some pair interaction is set
    SoftSphereDev pair[REP_TYPES][REP_TYPES];
    SoftSphereDev wall[REP_TYPES];
    int n_shape;
    const ShapeDev* shape;
    const unsigned char* type;  // [M] part type per node
    double* pos;                // [M][3] positions the forces are taken at
    int* cell;                  // [M] cell of each node
    int* cnt;                   // [ncell + 1] nodes per cell, then cell starts
    int* cursor;                // [ncell]
    int* bsum;                  // block sums of the scan
    int* list;                  // [M] node ids in cell order
    double* spos;               // [M][3] positions in cell order
    unsigned char* stype;       // [M] types in cell order
    void* frep;                 // [M][3] force, arithmetic type
    unsigned* status;           // the box's watchdog word (ST_OVERFLOW: a force out of range)
};

// ---- launchers (kernels.hip) ----------------------------------------------
// Which nodes a lattice launch updates.
enum : int {
    LB_ALL = 0,      // every node (coupling force read where the mask says so)
    LB_FREE = 1,     // only nodes whose touch bit (touch[parity]) is clear
    LB_TOUCHED = 2,  // only nodes whose touch bit is set; clears touch[parity] and the mask
};

struct LbLaunch {
    const BoxDev* boxes;   // device array
    const int2* work;      // device array (box, block) or nullptr for box 0
    int nblocks;
    int block;
    int parity;
    int remap;
    int precision;
    hipStream_t stream;
    int mode;              // LB_ALL, LB_FREE or LB_TOUCHED
    int obstacles;         // the boxes of the launch have obstacles
    int mrt;               // the boxes of the launch use the MRT collision
    int nt;                // population reads are non-temporal (all-node launches)
};
hipError_t launch_lb(const LbLaunch& L);

// Set touch[parity] bits of every lattice node inside the 2x2x2 stencil of any
// mesh node of the given objects (one workgroup per object).
hipError_t launch_mark(const void* objs, int nobj, int precision, size_t lds_bytes, int parity,
                       hipStream_t s);

struct MeshLaunch {
    const void* objs;      // device array of ObjDev<real>
    int nobj;
    int block;
    int parity;
    int precision;
    size_t lds_bytes;      // dynamic LDS per block (0 = each object's global scratch)
    size_t cpl_lds_bytes;  // scratch launch: dynamic LDS holding the coupling area (stencil
                           // bits, touched-node velocities and force sums); 0 = that
                           // area in the scratch too
    int mark_next;         // also mark the stencils of the new positions in
                           // touch[parity ^ 1] (split stepping)
    int conservative;      // some object of the launch uses the conservative force model
    hipStream_t stream;
    // split launches (work != null): split_lds of LDS, one workgroup per
    // (object, slice) in work (object index into objs, slice); the elements
    // launch, then the nodes launch
    const int2* work;
    int nwork;
    size_t split_lds;
    int lists;             // some box of the launch has the membrane kernel clear G
};
hipError_t launch_mesh(const MeshLaunch& L);

// Soft-sphere forces of one box into rep->frep (host copy `h` of the device
// descriptor `d` gives the sizes): bin, scan, scatter, order, force.
hipError_t launch_repulsion(const RepDev& h, const RepDev* d, const void* objs, int nobj, int precision,
                            hipStream_t s);

// Per-template LDS bytes of the mesh kernel.
size_t mesh_lds_bytes(int precision, int nv, int nt, int ne, int ucap, int ccap, int cons);
// Bytes of the coupling area alone (the part of the layout from `need` on).
size_t mesh_cpl_lds_bytes(int precision, int nv, int nt, int ne, int ucap, int ccap, int cons);
// Allow the LDS-resident mesh kernels to use up to `bytes` of dynamic LDS.
hipError_t mesh_set_max_lds(size_t bytes);

// FP64 diagnostics.  Lattice partials: per block [sum dev, jx, jy, jz, nonfinite];
// mesh partials: per object [0, m vx, m vy, m vz, nonfinite], stored after the
// lattice partials; final: out[0..4] lattice sums, out[5..9] mesh sums.
hipError_t launch_diag_lattice(const BoxDev* box_dev, int precision, int parity, double* partials,
                               int nblocks, hipStream_t s);
hipError_t launch_diag_mesh(const void* objs, int nobj, int precision, double* partials,
                            hipStream_t s);
hipError_t launch_diag_final(const double* partials, int nlat, int nmesh, double* out, hipStream_t s);

// plain device-to-device copy kernel of `bytes` (a multiple of 16)
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// conversions between the storage form and canonical FP64 arrays: full
// populations, or (deviations = 1) the deviations n_i - w_i rho0 exactly as
// stored
hipError_t launch_pops_to_f64(const BoxDev* box_dev, int N, int precision, int parity, double* out,
                              int deviations, hipStream_t s);
hipError_t launch_f64_to_pops(const BoxDev* box_dev, int N, int precision, int parity,
                              const double* in, int deviations, hipStream_t s);
hipError_t launch_moments(const BoxDev* box_dev, int N, int precision, int parity, double* rho,
                          double* u, hipStream_t s);

}  // namespace oif
