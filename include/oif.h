/*
 * oif.h -- C ABI of the MI355X (gfx950) coupled lattice-Boltzmann /
 * immersed-elastic-object step.
 *
 * Method: Cimrak, Gusenbauer, Jancigova, "An ESPResSo implementation of
 * elastic objects immersed in a fluid" -- Section "Method" (D3Q19 LB update,
 * eq. lbequation; IB point dynamics, eq. newton; drag coupling,
 * eq. dragforce, with linear interpolation of the fluid velocity and
 * distribution of the opposite force), Section "Elastic interactions"
 * (stretching, bending, local area, global area, volume forces) and
 * Section "Implementation details and OIF command description" (templates,
 * objects, analysis, customisation).
 *
 * Conventions shared by every call
 *   - Lattice units: grid spacing 1, time step 1.  Lattice node (i, j, k)
 *     sits at (i + 1/2, j + 1/2, k + 1/2); the box spans [0,nx)x[0,ny)x[0,nz).
 *   - D3Q19 ordering: 0 rest; 1/2 = +-x; 3/4 = +-y; 5/6 = +-z;
 *     7/8 = (1,1,0)/(-1,-1,0); 9/10 = (1,-1,0)/(-1,1,0);
 *     11/12 = (1,0,1)/(-1,0,-1); 13/14 = (1,0,-1)/(-1,0,1);
 *     15/16 = (0,1,1)/(0,-1,-1); 17/18 = (0,1,-1)/(0,-1,1).
 *   - Field layouts on the host: populations [19][nz][ny][nx] (x fastest),
 *     vector fields [3][nz][ny][nx], mesh arrays [node][3].
 *   - Collision: BGK with relaxation time tau, second-order equilibrium, Guo
 *     forcing with force density g + G (G = coupling force); fluid velocity
 *     u = (sum_i n_i e_i + F/2) / rho.  Drag: the mesh point feels
 *     -xi (v - u), the fluid receives +xi (v - u) with trilinear weights.
 *     Mesh update: symplectic Euler (v += F/m, then x += v).
 *   - Every call returns OIF_OK (0) or a negative error code; the message of
 *     the last error of a context is returned by oif_last_error.
 *   - Ownership: input arrays are copied during the call and stay the
 *     caller's; output arrays are caller-allocated host memory of the stated
 *     size.  Device memory is owned by the context, except population
 *     buffers the caller binds with oif_bind_device_buffers.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef OIF_H
#define OIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
/* The library is built with hidden symbol visibility; the calls declared
 * here are its only exports. */
#pragma GCC visibility push(default)

/* error codes */
#define OIF_OK 0
#define OIF_E_ARG (-1)         /* bad pointer, size, id range or non-finite parameter */
#define OIF_E_ID (-2)          /* ids must start at 0 and be consecutive */
#define OIF_E_MESH (-3)        /* mesh not closed/manifold or not inward-oriented */
#define OIF_E_STATE (-4)       /* call not valid in the current state */
#define OIF_E_NOMEM (-5)       /* device or host allocation failed */
#define OIF_E_HIP (-6)         /* a HIP runtime call failed */
#define OIF_E_NONFINITE (-7)   /* watchdog: NaN/Inf in populations or mesh state */
#define OIF_E_OVERFLOW (-8)    /* watchdog: fixed-point force accumulator out of range */
#define OIF_E_UNSUPPORTED (-9) /* configuration the library does not support */

/* precision forms of the lattice populations */
#define OIF_PREC_FP64 0          /* FP64 arithmetic and storage */
#define OIF_PREC_FP32 1          /* FP32 arithmetic, FP32 storage of deviations */
#define OIF_PREC_FP32_ST_FP16 2  /* FP32 arithmetic, FP16 storage of deviations x 2^s */
#define OIF_PREC_FP32_ST_BF16 3  /* FP32 arithmetic, BF16 storage of deviations */

/* stretching law ("Stretching force": neo-Hookean kappa(lambda), or kappa = 1) */
#define OIF_STRETCH_NEOHOOKE 0
#define OIF_STRETCH_LINEAR 1

/* Force models of a template.  PAPER: the bending, local-area and global-area
 * rules as printed ("Elastic interactions").  CONSERVATIVE: the same energies'
 * scales with directions that exert no net force and no torque on any hinge or
 * triangle: bending as -grad[kb hbar (theta - theta0)^2 / (2 theta0)] (hbar =
 * mean relaxed wing height of the hinge; the wings move along their normals by
 * 1/h, the edge vertices take the rest split by where the wings' feet lie on
 * the edge), local and global area along t_v / t_rms (centroid-to-vertex
 * vectors over their RMS length) instead of unit vectors.  Both coincide on
 * symmetric hinges and equilateral triangles; stretching and volume forces are
 * the same in both. */
#define OIF_FORCES_PAPER 0
#define OIF_FORCES_CONSERVATIVE 1

typedef struct oif_ctx oif_ctx;
typedef struct oif_batch oif_batch;

/* Fluid box ("Method"; the lbfluid parameters of the paper's example script).
 *   nx, ny, nz      lattice size, each in [1, 4096], nx*ny*nz rounded up to a
 *                   multiple of 64 below 2^31 / 19
 *   walls_z         1: halfway bounce-back walls at z = 0 and z = nz (needs nz >= 2)
 *   tau             BGK relaxation time, > 1/2 (kinematic viscosity (tau - 1/2)/3)
 *   rho0            rest density, > 0; the fluid starts at rest at rho0
 *   body_force      uniform force density g
 *   friction        drag coefficient xi of eq. dragforce, >= 0
 *   precision       OIF_PREC_*
 *   fp16_scale_exp  FP16 storage: deviations n_i - w_i rho0 are stored times
 *                   2^fp16_scale_exp, in [0, 24]
 *   fixed_point_exp FP32 modes: the coupling force density is accumulated in
 *                   int64 with resolution 2^-fixed_point_exp, in [16, 56];
 *                   each value added must lie below 2^(55 - fixed_point_exp)
 *                   (else OIF_E_OVERFLOW), so up to 256 of them can meet in
 *                   one lattice node without leaving the int64 range
 *                   (the FP64 mode accumulates each component as two int64
 *                   sums, of its multiples of 2^-30 and of the remainders in
 *                   units of 2^-80: exact and order-independent sums too, a
 *                   value rounded only below 2^-80, |value| < 2^25 with the
 *                   same room for 256 values)
 *   device          HIP device ordinal
 * Fill with oif_lattice_desc_init first; it sets tau 1, rho0 1, friction 0,
 * FP32, fp16_scale_exp 12, fixed_point_exp 40, device 0, sizes 0. */
typedef struct {
    int nx, ny, nz;
    int walls_z;
    double tau;
    double rho0;
    double body_force[3];
    double friction;
    int precision;
    int fp16_scale_exp;
    int fixed_point_exp;
    int device;
} oif_lattice_desc;

/* Elastic moduli of a template ("Elastic interactions"); 0 switches a force off. */
typedef struct {
    double ks, kb, kal, kag, kv;
    int stretch_law; /* OIF_STRETCH_* */
    int force_model; /* OIF_FORCES_* (0 = the paper's rules) */
} oif_moduli;

/* Object analysis (oif_object_analyze of the paper): origin = mean of the
 * mesh nodes, bounds = {xmin, xmax, ymin, ymax, zmin, zmax}, enclosed volume,
 * surface area, velocity = mean of the node velocities. */
typedef struct {
    double origin[3];
    double bounds[6];
    double volume;
    double area;
    double velocity[3];
} oif_analysis;

/* Counts and sizes (oif_info of the paper). */
typedef struct {
    int n_templates;
    int n_objects;
    int precision;
    int walls_z;
    long long n_nodes;
    long long n_mesh_nodes;
    long long steps_done;
    long long device_bytes;
    int lb_block;       /* tuned launch shapes in use */
    int mesh_block;
    int xcd_remap;
    int graph_steps;    /* steps per captured hipGraph, 0 = eager launches */
    long long max_lds;  /* LDS bytes per workgroup available to the membrane kernel */
    int lds_objects;    /* objects whose mesh is staged in LDS (the rest use global scratch) */
    int overlap;        /* 1 if untouched nodes are updated concurrently with the membrane kernel */
    int integrator;     /* OIF_INTEGRATOR_EULER or OIF_INTEGRATOR_VERLET */
    int lb_nontemporal; /* population reads of the lattice kernel: 1 non-temporal, 0 ordinary */
    int cpl_objects;    /* objects in the global scratch whose coupling area (stencil bits,
                           touched-node velocities, force sums) sits in LDS */
    long long cpl_lds_bytes; /* LDS bytes per workgroup of that coupling area (0: no such object) */
    int split_objects;  /* objects too large for LDS split over several workgroups each: triangles
                           and edges in slices, then the nodes in compact patches, with their
                           positions, the patch's forces and the coupling area in LDS */
    int split_workgroups; /* workgroups of each of the two split launches */
    long long split_lds_bytes; /* LDS bytes per workgroup of those launches (0: no such object) */
    int force_clear_by_membrane; /* see oif_set_force_clear */
} oif_info_t;

/* FP64 conservation diagnostics and watchdog state. */
typedef struct {
    double mass;              /* sum of rho over the lattice */
    double momentum_fluid[3]; /* sum over nodes of sum_i n_i e_i */
    double momentum_mesh[3];  /* sum over mesh nodes of m v */
    int nonfinite;            /* non-zero if any population or mesh value is NaN/Inf */
    int clamped;              /* non-zero if a stencil reached past a z-wall and was clamped */
    int overflow;             /* non-zero if a coupling force was out of fixed-point range */
} oif_diag;

/* Timing of one oif_step_timed call (HIP events on the streams the kernels run
 * on).  With overlap (see oif_set_overlap) lb_ms is the lattice launch over the
 * untouched nodes, which runs concurrently with the membrane kernel, and
 * lb_touched_ms the launch over the touched nodes after it. */
typedef struct {
    double total_ms;      /* first launch to last launch of the call */
    double lb_ms;         /* average duration of one lattice kernel launch */
    double mesh_ms;       /* average duration of one membrane/coupling kernel launch */
    int lb_launches;
    int mesh_launches;
    double lb_touched_ms; /* overlap only: lattice launch over the touched nodes */
    double mark_ms;       /* overlap only: marking of the touched nodes */
    int overlap;          /* 1 if the steps ran overlapped */
} oif_timing;

/* ---- lattice -------------------------------------------------------------- */

/* Fill d with defaults (see oif_lattice_desc).  Errors: OIF_E_ARG if d is NULL. */
int oif_lattice_desc_init(oif_lattice_desc* d);

/* Create a context: allocates the lattice on the device and sets the fluid
 * to rest at rho0 (oif_init + lbfluid of the paper).  *out receives the
 * context.  Errors: OIF_E_ARG (invalid desc), OIF_E_UNSUPPORTED (no gfx950
 * device), OIF_E_NOMEM, OIF_E_HIP. */
int oif_create(const oif_lattice_desc* desc, oif_ctx** out);

/* Release all device and host memory of the context.  NULL is accepted. */
int oif_destroy(oif_ctx* ctx);

/* Message of the context's last error ("" if none); owned by the context. */
const char* oif_last_error(const oif_ctx* ctx);

/* Run the context's work on the given hipStream_t (e.g. a PyTorch stream)
 * instead of its own stream; NULL restores the own stream.  The caller keeps
 * the stream alive while it is bound. */
int oif_bind_stream(oif_ctx* ctx, void* hip_stream);

/* Bytes of each of the context's two population buffers (*bytes). */
int oif_population_bytes(const oif_ctx* ctx, size_t* bytes);

/* Keep the context's two population buffers (the stored deviations of the
 * current and the next step, in the library's own tiled layout: opaque to the
 * caller) in caller-owned device memory, e.g. two tensors allocated by
 * PyTorch: f0 and f1 each of `bytes` >= oif_population_bytes, 256-byte
 * aligned, disjoint, device memory of the context's device, with no work
 * pending on them.  The current state is copied into them and the context's
 * own buffers are freed; both NULL copies the state back into buffers of the
 * context's own (bytes ignored).  While bound, the caller keeps the memory
 * alive and leaves it alone; the context never frees it.  Captured graphs are
 * dropped and batches holding the box take the new buffers at their next
 * step.  Binding again while bound moves the state into the new buffers; each
 * new buffer may be the one it replaces but must not otherwise overlap the
 * bound ones.  Errors: OIF_E_ARG (one NULL, too small, misaligned,
 * overlapping, or not device memory of the device; nothing changes),
 * OIF_E_NOMEM, OIF_E_HIP. */
int oif_bind_device_buffers(oif_ctx* ctx, void* f0, void* f1, size_t bytes);

/* ---- obstacles ---------------------------------------------------------------- */

/* Obstacles (the lbboundary shapes of the paper's simulation scripts,
 * "Implementation details"): every lattice node whose centre lies inside the
 * shape (faces included) becomes a solid node of a new boundary moving with
 * `velocity` (NULL = at rest); *id (may be NULL) receives its id, 1-based.  A
 * population that would stream into a solid node returns to its own node in
 * the opposite direction, less 6 w_i rho0 (e_i . u_wall): bounce-back from a
 * moving wall, so a moving boundary drives the fluid (a velocity inlet or a
 * sliding wall).  Solid nodes are not updated, report rho0 and the wall
 * velocity to the coupling and to oif_read_density/velocity, and take no share
 * of the spread coupling force.  A later boundary overwrites earlier ones
 * where they overlap; at most 255 per context.  The built-in z walls
 * (walls_z) are separate and act first.
 * Rhomboid: {corner + s a + t b + u c : s, t, u in [0, 1]}, the edge vectors
 * linearly independent.  Wall: the half-space n . x < dist with n = normal /
 * |normal|.  Each shape also bounds the soft-sphere wall interactions
 * (oif_set_wall_soft_sphere).  Errors: OIF_E_ARG (non-finite or degenerate
 * shape, non-finite velocity, 255 boundaries already; such a call changes
 * nothing), OIF_E_NOMEM, OIF_E_HIP. */
int oif_boundary_rhomboid(oif_ctx* ctx, const double corner[3], const double a[3], const double b[3],
                          const double c[3], const double velocity[3], int* id);
int oif_boundary_wall(oif_ctx* ctx, const double normal[3], double dist, const double velocity[3], int* id);

/* Remove all obstacles. */
int oif_boundary_clear(oif_ctx* ctx);

/* Boundary id of every node (0 = fluid): caller-allocated uint8 [N], layout
 * [z][y][x]. */
int oif_read_boundary(oif_ctx* ctx, uint8_t* out);

/* ---- templates and objects ------------------------------------------------ */

/* Register template tid (template creation of the paper).  nodes: nv x 3
 * coordinates, approximately centred at the origin; tris: nt x 3 node ids
 * whose normal AB x AC points INTO the object.  stretch (NULL = 1,1,1) scales
 * the coordinates per axis before the relaxed lengths, angles, wing heights,
 * triangle areas, total area and volume are computed (in FP64, on the host).
 * Ids start at 0 and are consecutive; a template cannot change once objects
 * exist.  Errors: OIF_E_ARG (also an unknown stretch law or force model),
 * OIF_E_ID, OIF_E_MESH (not closed, not manifold, inconsistent orientation,
 * or enclosed volume <= 0, i.e. outward normals), OIF_E_STATE. */
int oif_template_create(oif_ctx* ctx, int tid, const double* nodes, int nv, const int32_t* tris,
                        int nt, const double stretch[3], const oif_moduli* k);

/* Add object oid made from template tid (adding objects of the paper):
 * node positions = origin + R x_template, R = rot (row-major 3x3, NULL =
 * identity).  mass <= 0 means the default 1.  part_type (0..15, the part-type
 * of the paper's object command) selects the soft-sphere interactions of the
 * object's nodes.  Objects start at rest.  Errors: OIF_E_ARG, OIF_E_ID. */
int oif_object_add(oif_ctx* ctx, int oid, int tid, const double origin[3], const double rot[9],
                   double mass, int part_type);

/* R = Rz(rz) Ry(ry) Rx(rx): rotation by rx about x, then ry about y, then rz
 * about z (fixed axes), row-major. */
int oif_euler_to_rot(double rx, double ry, double rz, double R[9]);

/* The same external force on every node of object oid (object
 * customisation: force). */
int oif_object_set_force(oif_ctx* ctx, int oid, const double f[3]);

/* Translate object oid so that the mean of its nodes is at o (object
 * customisation: origin).  Errors: OIF_E_ARG for a non-finite o or
 * |o| > 1e6 (as in oif_object_add), or an unknown oid. */
int oif_object_set_origin(oif_ctx* ctx, int oid, const double o[3]);

/* Replace the node positions of object oid (object customisation:
 * mesh-nodes); x holds nv x 3 absolute coordinates. */
int oif_object_set_nodes(oif_ctx* ctx, int oid, const double* x);

/* ---- stepping ------------------------------------------------------------- */

/* Advance n_steps coupled steps (membrane forces, coupling, mesh update, LB
 * update), then run the FP64 watchdog.  Returns OIF_E_NONFINITE or
 * OIF_E_OVERFLOW if the watchdog trips (the state is kept for inspection).
 * Steps are replayed from captured hipGraphs when graph mode is on. */
int oif_step(oif_ctx* ctx, int n_steps);

/* Same as oif_step with eager launches bracketed by HIP events; fills t. */
int oif_step_timed(oif_ctx* ctx, int n_steps, oif_timing* t);

/* Graph mode: steps_per_graph > 0 captures that many steps (rounded up to an
 * even number) in one hipGraph and replays it; 0 launches eagerly. */
int oif_set_graph(oif_ctx* ctx, int steps_per_graph);

/* Collision operator.  Default: BGK with the relaxation time tau of the
 * lattice description (the paper requires only mass and momentum
 * conservation of the collision and defers its form to its LB references).
 * gamma = {shear, bulk, odd, even} selects the multiple-relaxation-time
 * operator of those references instead, in the orthogonal D3Q19 mode space:
 * mass kept, momentum + F, the traceless and trace parts of the stress
 * relaxed about rho/3 I + rho u u by gamma[0] and gamma[1] (force term
 * (1 + gamma)/2 (u F + F u), u = (j + F/2)/rho), the non-hydrodynamic
 * remainder scaled by gamma[2] / gamma[3] in its parts odd / even under
 * e -> -e.  Each factor must lie in (-1, 1) (OIF_E_ARG otherwise); the
 * kinematic viscosity is (1 + gamma[0]) / (6 (1 - gamma[0])), and all four
 * equal to 1 - 1/tau give the BGK operator.  gamma = NULL returns to BGK. */
int oif_set_mrt(oif_ctx* ctx, const double* gamma);

/* Soft-sphere repulsion, the object-object and object-wall collisions of the
 * paper's channel script ("inter type_a type_b soft-sphere a n cutoff
 * offset"): V(d) = a (d - offset)^-n for offset < d < offset + cutoff, zero
 * beyond, the force a n (d - offset)^-(n+1) pushing the partners apart.
 * oif_set_soft_sphere acts between any two distinct mesh nodes of part types
 * type_a and type_b (symmetric; the same type also within one object), at
 * the minimum-image distance in the periodic directions; every periodic box
 * length must be at least 2 (cutoff + offset).  oif_set_wall_soft_sphere acts
 * between the nodes of a part type and each obstacle shape (distance from the
 * node, wrapped into the box, to the shape's surface; no force on a node
 * inside a shape) and the walls z = 0 and z = nz when they are on.  The
 * forces are taken where the membrane forces are (step start, or after the
 * first half kick and drift with velocity Verlet) and added to each node's
 * total force; found through cell lists of the mesh nodes, summed in FP64 in
 * a fixed order.  a = 0 removes an interaction.  Types 0..15; a >= 0,
 * n > 0, cutoff > 0, offset >= 0, finite (OIF_E_ARG otherwise).  The
 * parameters are in lattice units (the paper's script values are in its own
 * units with time step 0.1). */
int oif_set_soft_sphere(oif_ctx* ctx, int type_a, int type_b, double a, double n, double cutoff,
                        double offset);
int oif_set_wall_soft_sphere(oif_ctx* ctx, int type, double a, double n, double cutoff, double offset);

/* Mesh integrator (eq. newton, time step 1).  EULER (default): forces and
 * drag from the positions and velocities at the start of the step, V += F/m,
 * then X += V.  VERLET, the velocity Verlet scheme of the paper's engine:
 * V_h = V + F_last/(2m), X += V_h, then membrane forces at the new positions,
 * the drag xi (V_h - u) with u interpolated there, V = V_h + F/(2m); the total
 * force F is carried into the next step (zero after switching integrators or
 * adding objects).  Overlapped stepping supports EULER only (OIF_E_STATE). */
#define OIF_INTEGRATOR_EULER 0
#define OIF_INTEGRATOR_VERLET 1
int oif_set_integrator(oif_ctx* ctx, int integrator);

/* The force carried by the VERLET integrator (total force of the last step,
 * 3 doubles per mesh node, object oid or -1 for all; zeros under EULER).
 * Writing it (VERLET only, else OIF_E_STATE; finite values) completes a
 * checkpoint restore together with oif_write_mesh and oif_write_populations. */
int oif_read_force(oif_ctx* ctx, int oid, double* F);
int oif_write_force(oif_ctx* ctx, int oid, const double* F);

/* Overlap (default off): the lattice nodes inside any mesh node's 2x2x2
 * stencil are marked (by the membrane kernel of the previous step); the lattice
 * update of all other nodes (which no coupling force can reach) then runs on a
 * second stream concurrently with the membrane/coupling kernel, and the marked
 * nodes are updated after it.  The result is identical to the sequential
 * order; 0 runs the step sequentially. */
int oif_set_overlap(oif_ctx* ctx, int on);

/* Launch shapes: lb_block in {64,128,256,512,1024}, mesh_block a multiple of
 * 64 in [64, 1024] (one workgroup per object: block sizes that let two objects
 * share a compute unit matter more than powers of two); xcd_remap 0/1 maps
 * consecutive lattice blocks to the same XCD.  Values < 0 keep the current
 * setting. */
int oif_set_launch(oif_ctx* ctx, int lb_block, int mesh_block, int xcd_remap);

/* Cache policy of the lattice kernel's population reads (the stored
 * populations of the collide-and-push update, Section "Method"): 1 issues
 * them as non-temporal loads (a value is dead once read, so these reads do not
 * displace the values just pushed, which the next step reads: this pays while
 * the two population buffers are not much larger than the last-level cache),
 * 0 as ordinary loads.  The results are identical either way.  Default: 1 when
 * the two buffers together hold at most 1 GiB, else 0; the autotuner measures
 * both.  OIF_E_ARG for a value other than 0 or 1. */
int oif_set_lb_loads(oif_ctx* ctx, int nontemporal);

/* Who clears the coupling force density G (the reaction of eq. dragforce
 * spread to the lattice, Section "Method").  G is kept per step parity.
 * 0 (default): the lattice kernel clears each node's G where it reads it.
 * 1: each membrane workgroup keeps the list of lattice nodes it added to and
 * zeroes them one step later, when the lattice kernel is done with them, so
 * the lattice kernel only reads G (its write traffic is the pushes alone);
 * the membrane kernel then writes what the lattice kernel no longer does.
 * Which is faster depends on the workload; the autotuner measures both.  The
 * results are identical either way, and the choice may change between any
 * two steps.  OIF_E_ARG for a value other than 0 or 1. */
int oif_set_force_clear(oif_ctx* ctx, int by_membrane);


/* Measured search of the launch shapes on this context's workload; the
 * choice is applied and, if cache_path is not NULL, stored there as JSON
 * keyed by device, precision and box shape (and read from it when present). */
int oif_autotune(oif_ctx* ctx, const char* cache_path);

/* ---- read-back / write ---------------------------------------------------- */

/* Full populations n_i in FP64, 19 * nx*ny*nz values, layout [19][nz][ny][nx]. */
int oif_read_populations(oif_ctx* ctx, double* out);

/* Overwrite the populations (same layout); the values are rounded to the
 * storage form of the context. */
int oif_write_populations(oif_ctx* ctx, const double* in);

/* The stored deviations n_i - w_i rho0 (same layout), in FP64, which holds
 * every storage form exactly (FP16 values unscaled).  Full populations near
 * w_i rho0 cannot carry the lowest bits of very small deviations (below about
 * 2^-31 rho0), so checkpoints use this pair: writing back what was read
 * restores the lattice state bit for bit in every precision form.  Written
 * values are rounded to the storage form. */
int oif_read_deviations(oif_ctx* ctx, double* out);
int oif_write_deviations(oif_ctx* ctx, const double* in);

/* Density rho [nz][ny][nx]. */
int oif_read_density(oif_ctx* ctx, double* out);

/* Velocity u = (sum_i n_i e_i + g/2) / rho, layout [3][nz][ny][nx]. */
int oif_read_velocity(oif_ctx* ctx, double* out);

/* Mesh positions (absolute, unwrapped) and velocities of object oid, or of
 * all objects concatenated in id order when oid = -1; X and V (either may be
 * NULL) hold n x 3 values. */
int oif_read_mesh(oif_ctx* ctx, int oid, double* X, double* V);

/* Overwrite positions and/or velocities (NULL keeps) of object oid or of all
 * objects (oid = -1); checkpoint restore. */
int oif_write_mesh(oif_ctx* ctx, int oid, const double* X, const double* V);

/* Object analysis (origin, bounds, volume, area, velocity). */
int oif_object_analyze(oif_ctx* ctx, int oid, oif_analysis* a);

int oif_info(oif_ctx* ctx, oif_info_t* info);

/* FP64 sums of mass and momentum and the watchdog flags of the current state. */
int oif_diagnostics(oif_ctx* ctx, oif_diag* d);

/* oif_diagnostics for callers that cannot allocate device memory (code under
 * stream capture elsewhere in the process, tight serving loops, harnesses that
 * forbid allocation): the same sums, bit for bit, with the partial sums in a
 * fixed 1 MiB device array that the library holds per device for the life of
 * the process, instead of memory the context allocates.  The call allocates
 * nothing and never re-creates the device mesh arrays: it returns
 * OIF_E_STATE while objects, templates or meshes changed since the last step
 * (step first), and OIF_E_ARG beyond 25952 objects (the array holds 5 doubles
 * per object and per lattice block).  All contexts on one device share that
 * array: calls that overlap in time on one device (several host threads)
 * race; every call overwrites what it reads, nothing needs clearing. */
int oif_diagnostics_noalloc(oif_ctx* ctx, oif_diag* d);

/* Number of distinct lattice nodes inside the 2x2x2 stencil of any mesh node
 * at the current positions (used for the byte model of the coupling). */
int oif_touched_nodes(oif_ctx* ctx, long long* count);

/* Measurement helper (not part of the method): bandwidth of a plain
 * 16-byte-per-thread device copy of `bytes` bytes (rounded down to a multiple
 * of 16) on `device`, averaged over `reps` launches, counting read plus write
 * (2 * bytes per launch).  Allocates and frees two buffers.  This is the
 * achievable-bandwidth reference for the lattice kernel's roofline and the
 * known-size kernel for scaling HBM byte counters.
 * Errors: OIF_E_ARG, OIF_E_UNSUPPORTED, OIF_E_NOMEM, OIF_E_HIP. */
int oif_copy_bandwidth(int device, long long bytes, int reps, double* gbps);

/* ---- batching form: many independent boxes advanced together --------------- */

/* Bind n existing contexts (same precision and device) into a batch: every
 * step launches one membrane/coupling kernel over all objects of all boxes
 * (largest meshes first) and one lattice kernel over all boxes' nodes.  The
 * contexts stay owned by the caller and must outlive the batch; stepping a
 * member context alone while the batch exists is allowed. */
int oif_batch_create(oif_ctx* const* boxes, int n, oif_batch** out);
int oif_batch_destroy(oif_batch* b);

/* Advance all boxes n_steps steps (graph-captured if oif_batch_set_graph was
 * given a positive count), then run each box's watchdog. */
int oif_batch_step(oif_batch* b, int n_steps);
int oif_batch_set_graph(oif_batch* b, int steps_per_graph);
int oif_batch_set_launch(oif_batch* b, int lb_block, int mesh_block, int xcd_remap);
int oif_batch_set_lb_loads(oif_batch* b, int nontemporal);

/* Persistent form (on = 1; default 0): every step is one launch of a kernel
 * whose workgroups, as many as fit on the device at once, take tasks from a
 * device list until it is done: the membrane, coupling and update of each
 * object (largest meshes first), then the lattice update of each block of
 * nodes of each box; a box's lattice blocks wait only for that box's
 * membranes, so the lattice update of boxes whose cells are done overlaps the
 * membranes of the others.  Same results as the launch-per-phase form (bit
 * for bit below FP64).  Boxes with obstacles or the MRT collision are not
 * supported in this form: stepping then returns OIF_E_UNSUPPORTED.  The launch
 * shapes are those of the membrane kernel (oif_batch_set_launch's mesh_block
 * is the workgroup size of both task kinds).  lattice_blocks_per_task: blocks
 * of mesh_block nodes that one lattice task updates (0: about three lattice
 * tasks per resident workgroup).  OIF_E_ARG for on outside {0, 1} or a
 * negative count. */
int oif_batch_set_persistent(oif_batch* b, int on, int lattice_blocks_per_task);
int oif_batch_autotune(oif_batch* b, const char* cache_path);
int oif_batch_step_timed(oif_batch* b, int n_steps, oif_timing* t);
const char* oif_batch_last_error(const oif_batch* b);

#pragma GCC visibility pop
#ifdef __cplusplus
}
#endif
#endif /* OIF_H */
