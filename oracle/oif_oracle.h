/*
 * oif_oracle.h -- plain FP64 CPU oracle for one coupled lattice-Boltzmann /
 * immersed-membrane time step (Cimrak, Gusenbauer, Jancigova: "An ESPResSo
 * implementation of elastic objects immersed in a fluid").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the tests, the smoke check and the bench's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * Conventions (the paper fixes none of them):
 *   D3Q19 ordering: 0 rest; 1/2 = +-x; 3/4 = +-y; 5/6 = +-z;
 *   7/8 = (1,1,0)/(-1,-1,0); 9/10 = (1,-1,0)/(-1,1,0);
 *   11/12 = (1,0,1)/(-1,0,-1); 13/14 = (1,0,-1)/(-1,0,1);
 *   15/16 = (0,1,1)/(0,-1,-1); 17/18 = (0,1,-1)/(0,-1,1).
 *   Populations are stored as full n_i (not deviations), layout
 *   [19][nz][ny][nx], x fastest.  Lattice node (i,j,k) sits at (i+1/2, j+1/2, k+1/2).
 *   Lattice units: grid spacing 1, time step 1.
 *   Triangles are stored with the normal AB x AC pointing into the object
 *   (template section of the paper).
 */
#ifndef OIF_ORACLE_H
#define OIF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* kappa(lambda) of the neo-Hookean stretching law ("Stretching force"). */
double orc_kappa(double lambda);

/* Undirected edges and hinges from a closed, consistently oriented triangle
 * list.  For every edge {u < v}: edge = (u, v); hinge = (A, B, C, D) where the
 * triangle T1 = hinge_tri[0] runs B -> C in its stored cyclic order and has the
 * third vertex A, and T2 = hinge_tri[1] is the other triangle on the edge with
 * third vertex D.  Arrays must hold 3*nt/2 entries.  Returns the edge count,
 * or -1 if an edge is not shared by exactly two oppositely oriented triangles. */
int orc_topology(int nv, int nt, const int* tri, int* edge, int* hinge, int* hinge_tri);

/* Triangle areas S[nt], total area, enclosed volume (inward orientation). */
void orc_geometry(int nv, const double* x, int nt, const int* tri, double* S,
                  double* area_total, double* volume);

/* Inner dihedral angle of a hinge (A, B, C, D) as defined for orc_topology. */
double orc_dihedral(const double* xa, const double* xb, const double* xc, const double* xd);

/* Relaxed values of a template from its node positions (after any stretch). */
void orc_relaxed(int nv, const double* x, int nt, const int* tri, int ne, const int* edge,
                 const int* hinge, double* L0, double* theta0, double* S0,
                 double* Sg0, double* V0);

/* Mean relaxed wing height of each hinge, (S(A,B,C) + S(D,C,B)) / |C - B|. */
void orc_wing_height(int nv, const double* x, int ne, const int* hinge, double* hbar);

/* Force models.  PAPER: the rules of "Elastic interactions" as printed.
 * CONSERVATIVE: bending as the gradient of kb hbar (theta - theta0)^2/(2 theta0)
 * and local/global area along t_v / t_rms, so that every hinge and triangle
 * exerts no net force and no torque; stretching and volume are unchanged. */
#define ORC_MODEL_PAPER 0
#define ORC_MODEL_CONSERVATIVE 1

/* Membrane forces of one object; ADDS into F[nv][3].
 * k = {ks, kb, kal, kag, kv}; linear != 0 selects kappa = 1; hbar (per edge,
 * from orc_wing_height) is read only by the conservative model. */
void orc_membrane_forces(int nv, const double* x, int nt, const int* tri, int ne,
                         const int* edge, const int* hinge, const double* L0,
                         const double* theta0, const double* S0, double Sg0, double V0,
                         const double* k, int linear, int model, const double* hbar, double* F);

/* Individual force families (same conventions), each ADDS into F. */
void orc_force_stretch(int nv, const double* x, int ne, const int* edge, const double* L0,
                       double ks, int linear, double* F);
void orc_force_bend(int nv, const double* x, int ne, const int* hinge, const double* theta0,
                    double kb, double* F);
void orc_force_local_area(int nv, const double* x, int nt, const int* tri, const double* S0,
                          double kal, double* F);
void orc_force_global_area(int nv, const double* x, int nt, const int* tri, double Sg0,
                           double kag, double* F);
void orc_force_volume(int nv, const double* x, int nt, const int* tri, double V0,
                      double kv, double* F);
/* conservative-model families */
void orc_force_bend_gradient(int nv, const double* x, int ne, const int* hinge,
                             const double* theta0, const double* hbar, double kb, double* F);
void orc_force_local_area_balanced(int nv, const double* x, int nt, const int* tri,
                                   const double* S0, double kal, double* F);
void orc_force_global_area_balanced(int nv, const double* x, int nt, const int* tri, double Sg0,
                                    double kag, double* F);

/* Lattice description. */
typedef struct {
    int nx, ny, nz;
    int walls_z;     /* halfway bounce-back walls at z = 0 and z = nz */
    double tau;      /* BGK relaxation time */
    double rho0;
    double g[3];     /* uniform body-force density */
    double xi;       /* friction coefficient of the drag coupling */
    /* obstacles (lbboundary of the paper's scripts), may be NULL: solid[N] =
     * 0 for fluid, k > 0 for a node of boundary k moving with velocity
     * wall_u[3 k .. 3 k + 2] */
    const unsigned char* solid;
    const double* wall_u;
    /* collision operator: ORC_BGK (relaxation time tau) or ORC_MRT, the
     * multiple-relaxation-time operator in the orthogonal mode space of the
     * D3Q19 set used by the paper's references: mass and momentum conserved,
     * the bulk (trace) and shear (traceless) parts of the stress relaxed by
     * gamma_bulk and gamma_shear, the odd and even non-hydrodynamic (ghost)
     * modes by gamma_odd and gamma_even */
    int collision;
    double gamma_shear, gamma_bulk, gamma_odd, gamma_even;
} orc_lattice;

#define ORC_BGK 0
#define ORC_MRT 1

/* Boundary shapes: set solid[p] = id for every node whose centre lies inside.
 * Rhomboid: {corner + s a + t b + u c : s, t, u in [0, 1]}.  Wall: the
 * half-space n.x < dist (n normalised). */
void orc_mark_rhomboid(const orc_lattice* L, unsigned char* solid, int id, const double* corner,
                       const double* a, const double* b, const double* c);
void orc_mark_wall(const orc_lattice* L, unsigned char* solid, int id, const double* normal,
                   double dist);

/* Density and velocity of every node, u = (sum n_i e_i + F/2) / rho with the
 * given force density field Fx (3*N, may be NULL for body force only); at a
 * solid node rho0 and the wall velocity. */
void orc_moments(const orc_lattice* L, const double* n, const double* Fx,
                 double* rho, double* u);

/* One collide + stream update of the whole lattice, n -> nout, with force
 * density g + G (G may be NULL).  A population streaming into a solid node
 * returns to its own node in the opposite direction, less
 * 6 w_i rho0 (e_i . u_wall) (bounce-back from a moving wall); solid nodes keep
 * their populations.  n and nout must not alias. */
void orc_lb_step(const orc_lattice* L, const double* n, const double* G, double* nout);

/* Trilinear stencil of a point: 8 node indices and weights.  Returns the number
 * of clamped corner indices (only with walls_z). */
int orc_stencil(const orc_lattice* L, const double* X, long* idx, double* w);

/* Drag coupling of one mesh point at X with velocity V: interpolates the node
 * velocity field u (3*N) at X, writes the force handed to the fluid,
 * drag = xi (V - u(X)), and ADDS its trilinear share to G (3*N) at fluid
 * nodes (a solid node takes none).  The point itself feels -drag.  Returns
 * the number of clamped corners. */
int orc_couple_point(const orc_lattice* L, const double* u, const double* X, const double* V,
                     double* G, double* drag);

/* Coupled system.  Mesh data of all objects is concatenated. */
typedef struct {
    int n_tmpl;
    const int* t_nv;        /* per template */
    const int* t_nt;
    const int* t_tri_off;   /* offset into tri (in triangles) */
    const int* tri;         /* concatenated [nt][3], template-local ids */
    const double* t_k;      /* [n_tmpl][5] ks kb kal kag kv */
    const int* t_linear;
    /* relaxed values, computed by orc_system_prepare */
    int n_obj;
    const int* o_tmpl;
    const int* o_node_off;  /* offset into X/V (in nodes) */
    const double* o_mass;
    const double* o_fext;   /* [n_obj][3] */
    const int* t_model;     /* per template ORC_MODEL_*, or NULL for all PAPER */
    int integrator;         /* ORC_EULER or ORC_VERLET (all objects) */
    /* soft-sphere repulsion (may be empty): part type per object, pair
     * interactions between mesh nodes of two types, and interactions of the
     * nodes of a type with every obstacle shape and the built-in z walls */
    const int* o_type;
    int n_pair;
    const struct orc_soft_sphere* pair;
    int n_wall;
    const struct orc_soft_sphere* wall;
    int n_shape;
    const struct orc_shape* shape;
} orc_mesh;

/* Soft-sphere interaction (the repulsion of the paper's scripts, "inter
 * type_a type_b soft-sphere a n cutoff offset"): V(d) = a (d - offset)^-n for
 * offset < d < offset + cutoff, zero beyond; the force a n (d - offset)^-(n+1)
 * pushes the two partners apart along the line joining them (for a wall:
 * along the line from the closest surface point).  Wall entries use type_a
 * only. */
typedef struct orc_soft_sphere {
    int type_a, type_b;
    double a, n, cutoff, offset;
} orc_soft_sphere;

/* Obstacle shapes for the wall repulsion: kind 0 = rhomboid {corner + s a +
 * t b + u c, s, t, u in [0, 1]}, kind 1 = wall, the half-space
 * normal . x < dist. */
typedef struct orc_shape {
    int kind;
    double corner[3], a[3], b[3], c[3];
    double normal[3], dist;
} orc_shape;

/* Distance from x to a shape's surface and the unit vector from the closest
 * surface point to x; returns 0 if x lies inside (or on) the shape. */
int orc_shape_distance(const orc_shape* sh, const double* x, double* dist, double* dir);


/* Mesh integrators (dt = 1).  EULER: forces from X_t, V_t; V += F/m, then
 * X += V.  VERLET (velocity Verlet, as in the paper's engine): V_h = V_t +
 * F_t/(2m), X_{t+1} = X_t + V_h, forces at X_{t+1} with the drag taken at
 * V_h, V_{t+1} = V_h + F_{t+1}/(2m); F_t is the total force of the previous
 * step (zero before the first step). */
#define ORC_EULER 0
#define ORC_VERLET 1

typedef struct orc_system orc_system;

/* Build a coupled system from template node coordinates (already stretched,
 * concatenated per template, t_x) and the object placements (X0 = absolute
 * initial positions of all mesh nodes).  Returns NULL on a mesh error. */
orc_system* orc_system_create(const orc_lattice* L, const orc_mesh* mesh,
                              const int* t_node_off, const double* t_x);
void orc_system_destroy(orc_system* s);

/* Advance n_steps coupled steps.  n: populations (19*N) in/out; X, V: mesh
 * positions/velocities (3*M) in/out.  diag (may be NULL) receives, for the LAST
 * step: [0] clamped stencil corners, [1..3] sum of elastic forces,
 * [4..6] sum of coupling forces on the mesh, [7..9] sum of external forces,
 * [10..12] sum of soft-sphere forces (13 doubles). */
int orc_system_run(orc_system* s, double* n, double* X, double* V, int n_steps, double* diag);

/* The total force of the last step on every mesh node (3*M): the force the
 * velocity Verlet integrator carries into the next step.  Read or replace it
 * (with X and V it is the integrator's whole state). */
void orc_system_get_force(const orc_system* s, double* F);
void orc_system_set_force(orc_system* s, const double* F);

/* Per-object geometry of the current positions: S_g[o], V[o]. */
void orc_system_geometry(orc_system* s, const double* X, double* Sg, double* Vol);

/* Elastic forces of all objects at positions X (overwrites F[3*M]). */
void orc_system_forces(orc_system* s, const double* X, double* F);

/* Soft-sphere forces on all mesh nodes at positions X (3*M), ADDED to F:
 * pairs of distinct nodes whose types interact (minimum-image distance in
 * the periodic directions), and the wall interactions (obstacle shapes at
 * their positions in the box, the planes z = 0 and z = nz with walls_z). */
void orc_system_repulsion(orc_system* s, const double* X, double* F);

/* Number of distinct lattice nodes inside any mesh node's 2x2x2 stencil. */
long orc_system_touched(orc_system* s, const double* X);

/* Host threads for the lattice sweeps (n > 0 sets them); returns the number
 * in use, 1 when built without OpenMP.  The results do not depend on it. */
int orc_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
