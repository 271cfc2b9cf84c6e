/*
 * oif_oracle.c -- plain FP64 CPU oracle of one coupled lattice-Boltzmann /
 * immersed-membrane time step, written from the paper (Cimrak, Gusenbauer,
 * Jancigova, "An ESPResSo implementation of elastic objects immersed in a
 * fluid", Sections "Method" and "Elastic interactions").
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes, links or
 * calls this file.  It is deliberately slow and serial so that every formula
 * can be checked against the paper by eye.  No blocking, fusion or
 * reordering beyond what the step definition states.
 *
 * Where the paper is silent or garbled, the readings used here are:
 *   - collision: single-relaxation-time BGK with relaxation time tau and the
 *     standard second-order equilibrium (the paper only requires mass and
 *     momentum conservation and defers the operator to its references); or,
 *     as an option, the multiple-relaxation-time operator of those references
 *     (relaxation in the orthogonal D3Q19 mode space, forcing as in the BGK
 *     case mode by mode), which equals BGK when every rate is 1 - 1/tau;
 *   - external force term f_i: Guo forcing, with the fluid velocity taken as
 *     u = (sum_i n_i e_i + F/2) / rho (equal to the paper's moment definition
 *     when F = 0);
 *   - drag: force on the mesh point -xi (v - u); the opposite force
 *     +xi (v - u) is spread to the fluid (eq. dragforce read so that the point
 *     relaxes towards the fluid velocity, momentum conserving);
 *   - interpolation and spreading: trilinear over the 8 surrounding nodes, each
 *     node weighted by the volume of the cuboid between the point and the
 *     diagonally opposite node (so spreading is the adjoint of interpolation);
 *   - the velocity interpolated is that of the populations at the start of the
 *     step, with half the body force only;
 *   - mesh integrator: symplectic Euler, V += F/m then X += V, time step 1;
 *     or, as an option, velocity Verlet (the integrator of the paper's
 *     engine) with the drag taken at the half-step velocity;
 *   - bending: theta = inner dihedral angle, n = inward unit normal of each
 *     triangle, the force on each wing vertex along its own triangle's normal,
 *     minus half the sum on each vertex of the shared edge;
 *   - volume force: along the outward normal (the stored normals point
 *     inward), one third of it on each vertex; the volume is the
 *     divergence-theorem sum over signed tetrahedra;
 *   - global area: per triangle, along the same centroid-to-vertex unit vector
 *     as the local area force, scaled by the object-global ratio;
 *   - collisions (the repulsion the paper's scripts set between part types
 *     and with the channel walls by name only): the soft-sphere potential
 *     a (d - offset)^-n inside offset < d < offset + cutoff, between any two
 *     distinct mesh nodes of interacting types (minimum-image distance) and
 *     between a node and each obstacle shape (distance to the shape's
 *     surface, no force on a node inside a shape).
 */
#include "oif_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Host threads of the two lattice sweeps (orc_moments, orc_lb_step).  Built
 * without OpenMP everything is serial.  Built with it, those sweeps split
 * their outer loop over threads: every node reads only the input arrays and
 * writes outputs no other node writes (its own moments; the populations it
 * pushes), so the result is bit for bit the serial one.  Everything else
 * (membrane forces, coupling, spreading) stays serial and ordered. */
int orc_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* D3Q19 velocity set, weights and opposites                                 */
/* ------------------------------------------------------------------------- */
static const int EV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int i) {
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite(int i) {
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------- */
static void sub3(const double* a, const double* b, double* r) {
    r[0] = a[0] - b[0];
    r[1] = a[1] - b[1];
    r[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------------- */
/* Stretching force: F_s = ks kappa(lambda) (dL / L0) n, with the            */
/* neo-Hookean kappa(lambda) = (lambda^0.5 + lambda^-2.5)/(lambda+lambda^-3) */
/* ------------------------------------------------------------------------- */
double orc_kappa(double lambda) {
    return (pow(lambda, 0.5) + pow(lambda, -2.5)) / (lambda + pow(lambda, -3.0));
}

/* ------------------------------------------------------------------------- */
/* Mesh topology                                                             */
/* ------------------------------------------------------------------------- */
typedef struct {
    int lo, hi;   /* undirected key */
    int from, to; /* directed edge as it appears in the triangle */
    int wing;     /* third vertex of the triangle */
    int t;        /* triangle id */
} dedge;

static int dedge_cmp(const void* pa, const void* pb) {
    const dedge* a = (const dedge*)pa;
    const dedge* b = (const dedge*)pb;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    /* put the lo -> hi direction first */
    int da = (a->from == a->lo) ? 0 : 1;
    int db = (b->from == b->lo) ? 0 : 1;
    return da - db;
}

int orc_topology(int nv, int nt, const int* tri, int* edge, int* hinge, int* hinge_tri) {
    int nd = 3 * nt;
    dedge* d = (dedge*)malloc(sizeof(dedge) * (size_t)nd);
    if (!d) return -1;
    for (int t = 0; t < nt; ++t) {
        for (int s = 0; s < 3; ++s) {
            int p = tri[3 * t + s];
            int q = tri[3 * t + (s + 1) % 3];
            int r = tri[3 * t + (s + 2) % 3];
            if (p < 0 || p >= nv || q < 0 || q >= nv || r < 0 || r >= nv || p == q) {
                free(d);
                return -1;
            }
            dedge* e = &d[3 * t + s];
            e->lo = p < q ? p : q;
            e->hi = p < q ? q : p;
            e->from = p;
            e->to = q;
            e->wing = r;
            e->t = t;
        }
    }
    qsort(d, (size_t)nd, sizeof(dedge), dedge_cmp);
    if (nd % 2) {
        free(d);
        return -1;
    }
    int ne = 0;
    for (int k = 0; k < nd; k += 2) {
        dedge* a = &d[k];
        dedge* b = &d[k + 1];
        /* each undirected edge exactly twice, once in each direction */
        if (a->lo != b->lo || a->hi != b->hi || a->from != a->lo || b->from != b->hi) {
            free(d);
            return -1;
        }
        if (k + 2 < nd && d[k + 2].lo == a->lo && d[k + 2].hi == a->hi) {
            free(d);
            return -1;
        }
        edge[2 * ne + 0] = a->lo;
        edge[2 * ne + 1] = a->hi;
        /* T1 runs B -> C (B = lo, C = hi), wing A; T2 has wing D */
        hinge[4 * ne + 0] = a->wing;
        hinge[4 * ne + 1] = a->from;
        hinge[4 * ne + 2] = a->to;
        hinge[4 * ne + 3] = b->wing;
        hinge_tri[2 * ne + 0] = a->t;
        hinge_tri[2 * ne + 1] = b->t;
        ++ne;
    }
    free(d);
    return ne;
}

/* ------------------------------------------------------------------------- */
/* Geometry: triangle areas, total surface, enclosed volume                  */
/* ------------------------------------------------------------------------- */
void orc_geometry(int nv, const double* x, int nt, const int* tri, double* S,
                  double* area_total, double* volume) {
    (void)nv;
    double A = 0.0, V = 0.0;
    const double* r0 = &x[0]; /* volume reference point: node 0 */
    for (int t = 0; t < nt; ++t) {
        const double* a = &x[3 * tri[3 * t + 0]];
        const double* b = &x[3 * tri[3 * t + 1]];
        const double* c = &x[3 * tri[3 * t + 2]];
        double ab[3], ac[3], N[3];
        sub3(b, a, ab);
        sub3(c, a, ac);
        cross3(ab, ac, N);
        double s = 0.5 * norm3(N);
        if (S) S[t] = s;
        A += s;
        /* signed tetrahedron (r0, a, b, c); with inward-oriented triangles
         * the sum of a~ . (b~ x c~) is -6 V */
        double at[3], bt[3], ct[3], bc[3];
        sub3(a, r0, at);
        sub3(b, r0, bt);
        sub3(c, r0, ct);
        cross3(bt, ct, bc);
        V += -dot3(at, bc) / 6.0;
    }
    if (area_total) *area_total = A;
    if (volume) *volume = V;
}

/* unit normal of triangle (a, b, c): AB x AC normalised (points inward for a
 * correctly stored triangle) */
static void unit_normal(const double* a, const double* b, const double* c, double* n) {
    double ab[3], ac[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    cross3(ab, ac, n);
    double l = norm3(n);
    n[0] /= l;
    n[1] /= l;
    n[2] /= l;
}

/* Inner dihedral angle of hinge (A, B, C, D): T1 = (A, B, C), T2 = (D, C, B)
 * in their stored cyclic orders.  theta = pi + atan2((n1 x n2) . e, n1 . n2)
 * with e the unit vector B -> C; a flat hinge gives pi, a convex one less. */
double orc_dihedral(const double* xa, const double* xb, const double* xc, const double* xd) {
    double n1[3], n2[3], e[3], m[3];
    unit_normal(xa, xb, xc, n1);
    unit_normal(xd, xc, xb, n2);
    sub3(xc, xb, e);
    double le = norm3(e);
    e[0] /= le;
    e[1] /= le;
    e[2] /= le;
    cross3(n1, n2, m);
    return M_PI + atan2(dot3(m, e), dot3(n1, n2));
}

void orc_relaxed(int nv, const double* x, int nt, const int* tri, int ne, const int* edge,
                 const int* hinge, double* L0, double* theta0, double* S0,
                 double* Sg0, double* V0) {
    for (int e = 0; e < ne; ++e) {
        double d[3];
        sub3(&x[3 * edge[2 * e + 1]], &x[3 * edge[2 * e + 0]], d);
        L0[e] = norm3(d);
        const int* h = &hinge[4 * e];
        theta0[e] = orc_dihedral(&x[3 * h[0]], &x[3 * h[1]], &x[3 * h[2]], &x[3 * h[3]]);
    }
    orc_geometry(nv, x, nt, tri, S0, Sg0, V0);
}

static double tri_area(const double* x, const int* tv);

void orc_wing_height(int nv, const double* x, int ne, const int* hinge, double* hbar) {
    (void)nv;
    for (int e = 0; e < ne; ++e) {
        const int* h = &hinge[4 * e];
        const int t1[3] = {h[0], h[1], h[2]}, t2[3] = {h[3], h[2], h[1]};
        double bc[3];
        sub3(&x[3 * h[2]], &x[3 * h[1]], bc);
        /* mean of the two wing heights 2 S / |BC| */
        hbar[e] = (tri_area(x, t1) + tri_area(x, t2)) / norm3(bc);
    }
}

/* ------------------------------------------------------------------------- */
/* Elastic forces ("Elastic interactions")                                   */
/* ------------------------------------------------------------------------- */

/* Stretching: each edge endpoint is pulled towards (L > L0) or pushed away
 * from (L < L0) the other with magnitude ks kappa(lambda) (L - L0)/L0. */
void orc_force_stretch(int nv, const double* x, int ne, const int* edge, const double* L0,
                       double ks, int linear, double* F) {
    (void)nv;
    if (ks == 0.0) return;
    for (int e = 0; e < ne; ++e) {
        int a = edge[2 * e], b = edge[2 * e + 1];
        double d[3];
        sub3(&x[3 * b], &x[3 * a], d);
        double L = norm3(d);
        double lam = L / L0[e];
        double kap = linear ? 1.0 : orc_kappa(lam);
        double f = ks * kap * (L - L0[e]) / L0[e];
        for (int c = 0; c < 3; ++c) {
            F[3 * a + c] += f * d[c] / L;
            F[3 * b + c] -= f * d[c] / L;
        }
    }
}

/* Bending: F_b = kb (theta - theta0)/theta0 n on each wing vertex along the
 * unit (inward) normal of its own triangle; each vertex of the shared edge
 * receives minus half the sum of the two wing forces. */
void orc_force_bend(int nv, const double* x, int ne, const int* hinge, const double* theta0,
                    double kb, double* F) {
    (void)nv;
    if (kb == 0.0) return;
    for (int e = 0; e < ne; ++e) {
        int A = hinge[4 * e], B = hinge[4 * e + 1], C = hinge[4 * e + 2], D = hinge[4 * e + 3];
        double n1[3], n2[3];
        unit_normal(&x[3 * A], &x[3 * B], &x[3 * C], n1);
        unit_normal(&x[3 * D], &x[3 * C], &x[3 * B], n2);
        double theta = orc_dihedral(&x[3 * A], &x[3 * B], &x[3 * C], &x[3 * D]);
        double f = kb * (theta - theta0[e]) / theta0[e];
        for (int c = 0; c < 3; ++c) {
            F[3 * A + c] += f * n1[c];
            F[3 * D + c] += f * n2[c];
            F[3 * B + c] -= 0.5 * f * (n1[c] + n2[c]);
            F[3 * C + c] -= 0.5 * f * (n1[c] + n2[c]);
        }
    }
}

/* Bending in gradient form: F = -grad E per hinge with
 * E = kb hbar (theta - theta0)^2 / (2 theta0), hbar the hinge's mean relaxed
 * wing height (orc_wing_height).  Gradient of the inner dihedral angle: moving
 * a wing vertex by d along its own triangle's inward normal turns that
 * triangle about the shared edge by d / h (h = the vertex's distance from the
 * edge line) and makes the hinge more convex, so grad_A theta = -n1 / h_A and
 * grad_D theta = -n2 / h_D; in-plane moves of a wing do not change theta.
 * With the feet of A and D on the edge at B + a (C - B), the edge vertices
 * take grad_B = -(1 - a_A) grad_A - (1 - a_D) grad_D and
 * grad_C = -a_A grad_A - a_D grad_D, which makes the gradient sum to zero
 * and carry no torque (theta is invariant under rigid motions).  On a
 * symmetric hinge (a = 1/2, h_A = h_D = hbar) this is the paper's rule with
 * its magnitude kb (theta - theta0)/theta0. */
void orc_force_bend_gradient(int nv, const double* x, int ne, const int* hinge,
                             const double* theta0, const double* hbar, double kb, double* F) {
    (void)nv;
    if (kb == 0.0) return;
    for (int e = 0; e < ne; ++e) {
        int A = hinge[4 * e], B = hinge[4 * e + 1], C = hinge[4 * e + 2], D = hinge[4 * e + 3];
        double n1[3], n2[3], bc[3], ba[3], bd[3], ca[3], cd[3];
        unit_normal(&x[3 * A], &x[3 * B], &x[3 * C], n1);
        unit_normal(&x[3 * D], &x[3 * C], &x[3 * B], n2);
        sub3(&x[3 * C], &x[3 * B], bc);
        sub3(&x[3 * A], &x[3 * B], ba);
        sub3(&x[3 * D], &x[3 * B], bd);
        double L2 = dot3(bc, bc);
        double aA = dot3(ba, bc) / L2, aD = dot3(bd, bc) / L2;
        cross3(ba, bc, ca);
        cross3(bd, bc, cd);
        double hA = norm3(ca) / sqrt(L2), hD = norm3(cd) / sqrt(L2);
        double theta = orc_dihedral(&x[3 * A], &x[3 * B], &x[3 * C], &x[3 * D]);
        double dEdt = kb * hbar[e] * (theta - theta0[e]) / theta0[e];
        for (int c = 0; c < 3; ++c) {
            double gA = -n1[c] / hA, gD = -n2[c] / hD;
            double gB = -(1.0 - aA) * gA - (1.0 - aD) * gD;
            double gC = -aA * gA - aD * gD;
            F[3 * A + c] -= dEdt * gA;
            F[3 * B + c] -= dEdt * gB;
            F[3 * C + c] -= dEdt * gC;
            F[3 * D + c] -= dEdt * gD;
        }
    }
}

/* Centroid-to-vertex directions of triangle t.  balanced = 0: unit vectors,
 * the paper's w.  balanced = 1: t_v / t_rms with t_rms^2 = (|t_a|^2 + |t_b|^2
 * + |t_c|^2) / 3; these sum to zero and are parallel to t_v, so forces along
 * them carry no net force and no torque about the centroid, and on an
 * equilateral triangle they are the unit vectors. */
static void tri_dirs(const double* x, const int* tv, int balanced, double w[3][3]) {
    double cen[3];
    for (int c = 0; c < 3; ++c)
        cen[c] = (x[3 * tv[0] + c] + x[3 * tv[1] + c] + x[3 * tv[2] + c]) / 3.0;
    double ms = 0.0;
    for (int s = 0; s < 3; ++s) {
        sub3(&x[3 * tv[s]], cen, w[s]);
        ms += dot3(w[s], w[s]) / 3.0;
    }
    for (int s = 0; s < 3; ++s) {
        double l = balanced ? sqrt(ms) : norm3(w[s]);
        for (int c = 0; c < 3; ++c) w[s][c] /= l;
    }
}

static void tri_w(const double* x, const int* tv, double w[3][3]) { tri_dirs(x, tv, 0, w); }

static double tri_area(const double* x, const int* tv) {
    double ab[3], ac[3], N[3];
    sub3(&x[3 * tv[1]], &x[3 * tv[0]], ab);
    sub3(&x[3 * tv[2]], &x[3 * tv[0]], ac);
    cross3(ab, ac, N);
    return 0.5 * norm3(N);
}

/* Local area: F_al = -kal (S - S0)/S w at each vertex. */
void orc_force_local_area(int nv, const double* x, int nt, const int* tri, const double* S0,
                          double kal, double* F) {
    (void)nv;
    if (kal == 0.0) return;
    for (int t = 0; t < nt; ++t) {
        const int* tv = &tri[3 * t];
        double S = tri_area(x, tv);
        double w[3][3];
        tri_w(x, tv, w);
        double coef = -kal * (S - S0[t]) / S;
        for (int s = 0; s < 3; ++s)
            for (int c = 0; c < 3; ++c) F[3 * tv[s] + c] += coef * w[s][c];
    }
}

/* Global area: F_ag = -kag (Sg - Sg0)/Sg w, applied per triangle to its
 * vertices with the local centroid-to-vertex direction. */
void orc_force_global_area(int nv, const double* x, int nt, const int* tri, double Sg0,
                           double kag, double* F) {
    if (kag == 0.0) return;
    double Sg;
    orc_geometry(nv, x, nt, tri, NULL, &Sg, NULL);
    double coef = -kag * (Sg - Sg0) / Sg;
    for (int t = 0; t < nt; ++t) {
        const int* tv = &tri[3 * t];
        double w[3][3];
        tri_w(x, tv, w);
        for (int s = 0; s < 3; ++s)
            for (int c = 0; c < 3; ++c) F[3 * tv[s] + c] += coef * w[s][c];
    }
}

/* Local and global area along the balanced directions t_v / t_rms (see
 * tri_dirs): the same magnitudes as the paper's rules, no net force or torque
 * on any triangle. */
void orc_force_local_area_balanced(int nv, const double* x, int nt, const int* tri,
                                   const double* S0, double kal, double* F) {
    (void)nv;
    if (kal == 0.0) return;
    for (int t = 0; t < nt; ++t) {
        const int* tv = &tri[3 * t];
        double S = tri_area(x, tv);
        double w[3][3];
        tri_dirs(x, tv, 1, w);
        double coef = -kal * (S - S0[t]) / S;
        for (int s = 0; s < 3; ++s)
            for (int c = 0; c < 3; ++c) F[3 * tv[s] + c] += coef * w[s][c];
    }
}

void orc_force_global_area_balanced(int nv, const double* x, int nt, const int* tri, double Sg0,
                                    double kag, double* F) {
    if (kag == 0.0) return;
    double Sg;
    orc_geometry(nv, x, nt, tri, NULL, &Sg, NULL);
    double coef = -kag * (Sg - Sg0) / Sg;
    for (int t = 0; t < nt; ++t) {
        const int* tv = &tri[3 * t];
        double w[3][3];
        tri_dirs(x, tv, 1, w);
        for (int s = 0; s < 3; ++s)
            for (int c = 0; c < 3; ++c) F[3 * tv[s] + c] += coef * w[s][c];
    }
}

/* Volume: per triangle F_v = -kv (V - V0)/V0 S n_out, one third to each vertex. */
void orc_force_volume(int nv, const double* x, int nt, const int* tri, double V0,
                      double kv, double* F) {
    if (kv == 0.0) return;
    double V;
    orc_geometry(nv, x, nt, tri, NULL, NULL, &V);
    double coef = -kv * (V - V0) / V0;
    for (int t = 0; t < nt; ++t) {
        const int* tv = &tri[3 * t];
        double n_in[3];
        unit_normal(&x[3 * tv[0]], &x[3 * tv[1]], &x[3 * tv[2]], n_in);
        double S = tri_area(x, tv);
        for (int s = 0; s < 3; ++s)
            for (int c = 0; c < 3; ++c) F[3 * tv[s] + c] += coef * S * (-n_in[c]) / 3.0;
    }
}

void orc_membrane_forces(int nv, const double* x, int nt, const int* tri, int ne,
                         const int* edge, const int* hinge, const double* L0,
                         const double* theta0, const double* S0, double Sg0, double V0,
                         const double* k, int linear, int model, const double* hbar, double* F) {
    orc_force_stretch(nv, x, ne, edge, L0, k[0], linear, F);
    if (model == ORC_MODEL_CONSERVATIVE) {
        orc_force_bend_gradient(nv, x, ne, hinge, theta0, hbar, k[1], F);
        orc_force_local_area_balanced(nv, x, nt, tri, S0, k[2], F);
        orc_force_global_area_balanced(nv, x, nt, tri, Sg0, k[3], F);
    } else {
        orc_force_bend(nv, x, ne, hinge, theta0, k[1], F);
        orc_force_local_area(nv, x, nt, tri, S0, k[2], F);
        orc_force_global_area(nv, x, nt, tri, Sg0, k[3], F);
    }
    orc_force_volume(nv, x, nt, tri, V0, k[4], F);
}

/* ------------------------------------------------------------------------- */
/* Lattice Boltzmann ("Method", eq. lbequation and the moment definitions)   */
/* ------------------------------------------------------------------------- */
static long node_index(const orc_lattice* L, int x, int y, int z) {
    return ((long)z * L->ny + y) * L->nx + x;
}

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

void orc_moments(const orc_lattice* L, const double* n, const double* Fx, double* rho,
                 double* u) {
    long N = (long)L->nx * L->ny * L->nz;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        if (L->solid && L->solid[p]) {
            if (rho) rho[p] = L->rho0;
            if (u)
                for (int c = 0; c < 3; ++c) u[c * N + p] = L->wall_u[3 * L->solid[p] + c];
            continue;
        }
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 19; ++i) {
            double ni = n[i * N + p];
            r += ni;
            for (int c = 0; c < 3; ++c) j[c] += ni * EV[i][c];
        }
        double F[3];
        for (int c = 0; c < 3; ++c) F[c] = L->g[c] + (Fx ? Fx[c * N + p] : 0.0);
        if (rho) rho[p] = r;
        if (u)
            for (int c = 0; c < 3; ++c) u[c * N + p] = (j[c] + 0.5 * F[c]) / r;
    }
}

/* BGK collision with Guo forcing of one node's populations nn[19] under the
 * force density F: post[i] = n_i - (n_i - n_i^eq)/tau + S_i. */
static void collide_bgk(const orc_lattice* L, const double* nn, const double* F, double* post) {
    double tau = L->tau;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        rho += nn[i];
        for (int c = 0; c < 3; ++c) j[c] += nn[i] * EV[i][c];
    }
    double u[3];
    for (int c = 0; c < 3; ++c) u[c] = (j[c] + 0.5 * F[c]) / rho;
    double usq = dot3(u, u);
    for (int i = 0; i < 19; ++i) {
        double e[3] = {EV[i][0], EV[i][1], EV[i][2]};
        double eu = dot3(e, u);
        double w = weight(i);
        /* second-order equilibrium */
        double neq = w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
        /* Guo source term */
        double src = 0.0;
        for (int c = 0; c < 3; ++c) src += (3.0 * (e[c] - u[c]) + 9.0 * eu * e[c]) * F[c];
        src *= (1.0 - 0.5 / tau) * w;
        post[i] = nn[i] - (nn[i] - neq) / tau + src;
    }
}

/* The orthogonal D3Q19 mode basis of the multiple-relaxation-time operator:
 * basis vector k evaluated at velocity e_i.  k = 0 density; 1-3 momentum;
 * 4 bulk stress (trace); 5-9 shear stress (traceless); 10-15 odd and 16-18
 * even non-hydrodynamic ("ghost") modes.  sum_i w_i b_k(e_i) b_l(e_i) = 0 for
 * k != l. */
static double mode_basis(int k, int i) {
    double x = EV[i][0], y = EV[i][1], z = EV[i][2];
    double c2 = x * x + y * y + z * z;
    switch (k) {
        case 0: return 1.0;
        case 1: return x;
        case 2: return y;
        case 3: return z;
        case 4: return c2 - 1.0;
        case 5: return 3.0 * x * x - c2;
        case 6: return y * y - z * z;
        case 7: return x * y;
        case 8: return x * z;
        case 9: return y * z;
        case 10: return (3.0 * c2 - 5.0) * x;
        case 11: return (3.0 * c2 - 5.0) * y;
        case 12: return (3.0 * c2 - 5.0) * z;
        case 13: return (y * y - z * z) * x;
        case 14: return (z * z - x * x) * y;
        case 15: return (x * x - y * y) * z;
        case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
        case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
        default: return (2.0 * c2 - 3.0) * (y * y - z * z);
    }
}

/* Multiple-relaxation-time collision of one node under the force density F.
 * Modes m_k = sum_i b_k(e_i) n_i.  Density is kept and the momentum gains F.
 * The stress modes relax towards their equilibrium values (those of the
 * second-order equilibrium, rho u u + rho c_s^2 I with u = (j + F/2)/rho) and
 * receive the force term of the same form as in the BGK case:
 *   m_k* = m_k^eq + gamma_k (m_k - m_k^eq) + (1 + gamma_k)/2 phi_k,
 * phi_k the mode k of the tensor u F + F u, gamma_k = gamma_bulk (k = 4) or
 * gamma_shear (5-9).  Ghost modes (equilibrium zero) become gamma m_k.  Back
 * to populations: n_i* = w_i sum_k b_k(e_i) m_k* / (sum_l w_l b_k(e_l)^2). */
static void collide_mrt(const orc_lattice* L, const double* nn, const double* F, double* post) {
    double m[19];
    for (int k = 0; k < 19; ++k) {
        m[k] = 0.0;
        for (int i = 0; i < 19; ++i) m[k] += mode_basis(k, i) * nn[i];
    }
    double rho = m[0];
    double u[3];
    for (int c = 0; c < 3; ++c) u[c] = (m[1 + c] + 0.5 * F[c]) / rho;
    /* equilibrium stress Pi_ab = rho/3 delta_ab + rho u_a u_b and force
     * tensor Phi_ab = u_a F_b + F_a u_b, mapped to modes 4-9 the way the
     * populations' second moments are: m4 = tr - rho, m5 = 3 xx - tr,
     * m6 = yy - zz, m7 = xy, m8 = xz, m9 = yz */
    double Pi[3][3], Phi[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            Pi[a][b] = rho * u[a] * u[b] + (a == b ? rho / 3.0 : 0.0);
            Phi[a][b] = u[a] * F[b] + F[a] * u[b];
        }
    double trPi = Pi[0][0] + Pi[1][1] + Pi[2][2], trPhi = Phi[0][0] + Phi[1][1] + Phi[2][2];
    double meq[10], phi[10];
    meq[4] = trPi - rho;
    meq[5] = 3.0 * Pi[0][0] - trPi;
    meq[6] = Pi[1][1] - Pi[2][2];
    meq[7] = Pi[0][1];
    meq[8] = Pi[0][2];
    meq[9] = Pi[1][2];
    phi[4] = trPhi;
    phi[5] = 3.0 * Phi[0][0] - trPhi;
    phi[6] = Phi[1][1] - Phi[2][2];
    phi[7] = Phi[0][1];
    phi[8] = Phi[0][2];
    phi[9] = Phi[1][2];
    double ms[19];
    ms[0] = m[0];
    for (int c = 0; c < 3; ++c) ms[1 + c] = m[1 + c] + F[c];
    for (int k = 4; k <= 9; ++k) {
        double g = (k == 4) ? L->gamma_bulk : L->gamma_shear;
        ms[k] = meq[k] + g * (m[k] - meq[k]) + 0.5 * (1.0 + g) * phi[k];
    }
    for (int k = 10; k <= 15; ++k) ms[k] = L->gamma_odd * m[k];
    for (int k = 16; k <= 18; ++k) ms[k] = L->gamma_even * m[k];
    for (int i = 0; i < 19; ++i) {
        double v = 0.0;
        for (int k = 0; k < 19; ++k) {
            double norm = 0.0;
            for (int l = 0; l < 19; ++l) norm += weight(l) * mode_basis(k, l) * mode_basis(k, l);
            v += mode_basis(k, i) * ms[k] / norm;
        }
        post[i] = weight(i) * v;
    }
}

void orc_lb_step(const orc_lattice* L, const double* n, const double* G, double* nout) {
    long N = (long)L->nx * L->ny * L->nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < L->nz; ++z)
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                long p = node_index(L, x, y, z);
                if (L->solid && L->solid[p]) {  /* obstacle node: not updated */
                    for (int i = 0; i < 19; ++i) nout[i * N + p] = n[i * N + p];
                    continue;
                }
                double F[3];
                for (int c = 0; c < 3; ++c) F[c] = L->g[c] + (G ? G[c * N + p] : 0.0);
                double nn[19], post[19];
                for (int i = 0; i < 19; ++i) nn[i] = n[i * N + p];
                if (L->collision == ORC_MRT) collide_mrt(L, nn, F, post);
                else collide_bgk(L, nn, F, post);
                for (int i = 0; i < 19; ++i) {
                    double e[3] = {EV[i][0], EV[i][1], EV[i][2]};
                    double w = weight(i);
                    double ns = post[i];
                    /* propagation to x + e_i */
                    int xd = wrap(x + EV[i][0], L->nx);
                    int yd = wrap(y + EV[i][1], L->ny);
                    int zd = z + EV[i][2];
                    if (L->walls_z && (zd < 0 || zd >= L->nz)) {
                        /* halfway bounce-back: the population returns to its
                         * own node in the opposite direction */
                        nout[opposite(i) * N + p] = ns;
                    } else {
                        zd = wrap(zd, L->nz);
                        long q = node_index(L, xd, yd, zd);
                        int b = L->solid ? L->solid[q] : 0;
                        if (b) {
                            /* bounce-back from an obstacle moving with u_w:
                             * n_opp(i)(x) = n_i*(x) - 2 w_i rho0 (e_i . u_w) / c_s^2 */
                            double euw = dot3(e, &L->wall_u[3 * b]);
                            nout[opposite(i) * N + p] = ns - 6.0 * w * L->rho0 * euw;
                        } else {
                            nout[i * N + q] = ns;
                        }
                    }
                }
            }
}

/* ------------------------------------------------------------------------- */
/* Coupling ("Immersed Boundary method", eq. dragforce and what follows)     */
/* ------------------------------------------------------------------------- */
int orc_stencil(const orc_lattice* L, const double* X, long* idx, double* w) {
    int dims[3] = {L->nx, L->ny, L->nz};
    int i0[3];
    double phi[3];
    for (int c = 0; c < 3; ++c) {
        double s = X[c] - 0.5; /* nodes sit at cell centres */
        double f = floor(s);
        i0[c] = (int)f;
        phi[c] = s - f;
    }
    int clamped = 0;
    int k = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int d[3] = {dx, dy, dz};
                int ii[3];
                double ww = 1.0;
                for (int c = 0; c < 3; ++c) {
                    ii[c] = i0[c] + d[c];
                    ww *= d[c] ? phi[c] : 1.0 - phi[c];
                }
                ii[0] = wrap(ii[0], dims[0]);
                ii[1] = wrap(ii[1], dims[1]);
                if (L->walls_z) {
                    if (ii[2] < 0) {
                        ii[2] = 0;
                        ++clamped;
                    } else if (ii[2] >= dims[2]) {
                        ii[2] = dims[2] - 1;
                        ++clamped;
                    }
                } else {
                    ii[2] = wrap(ii[2], dims[2]);
                }
                idx[k] = node_index(L, ii[0], ii[1], ii[2]);
                w[k] = ww;
                ++k;
            }
    return clamped;
}

int orc_couple_point(const orc_lattice* L, const double* u, const double* X, const double* V,
                     double* G, double* drag) {
    long N = (long)L->nx * L->ny * L->nz;
    long idx[8];
    double w[8];
    int clamped = orc_stencil(L, X, idx, w);
    /* fluid velocity at the point: linear interpolation from the 8 nodes */
    double uj[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 8; ++k)
        for (int c = 0; c < 3; ++c) uj[c] += w[k] * u[c * N + idx[k]];
    /* xi (v - u): the force handed to the fluid; the point feels its opposite */
    for (int c = 0; c < 3; ++c) drag[c] = L->xi * (V[c] - uj[c]);
    /* distributed to the same 8 nodes with the same weights (fluid nodes only) */
    for (int k = 0; k < 8; ++k) {
        if (L->solid && L->solid[idx[k]]) continue;
        for (int c = 0; c < 3; ++c) G[c * N + idx[k]] += w[k] * drag[c];
    }
    return clamped;
}

/* ------------------------------------------------------------------------- */
/* Obstacle shapes (the lbboundary shapes of the paper's scripts)            */
/* ------------------------------------------------------------------------- */

/* Rhomboid: solve (x - corner) = s a + t b + u c by Cramer's rule; the node
 * is inside when s, t, u all lie in [0, 1]. */
void orc_mark_rhomboid(const orc_lattice* L, unsigned char* solid, int id, const double* corner,
                       const double* a, const double* b, const double* c) {
    double bc[3], ca[3], ab[3];
    cross3(b, c, bc);
    cross3(c, a, ca);
    cross3(a, b, ab);
    double det = dot3(a, bc);
    for (int z = 0; z < L->nz; ++z)
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                double r[3] = {x + 0.5 - corner[0], y + 0.5 - corner[1], z + 0.5 - corner[2]};
                double s = dot3(r, bc) / det, t = dot3(r, ca) / det, u = dot3(r, ab) / det;
                if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0)
                    solid[node_index(L, x, y, z)] = (unsigned char)id;
            }
}

/* Wall: the half-space whose signed distance n.x - dist (n normalised) is
 * negative. */
void orc_mark_wall(const orc_lattice* L, unsigned char* solid, int id, const double* normal,
                   double dist) {
    double len = norm3(normal);
    for (int z = 0; z < L->nz; ++z)
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                double r[3] = {x + 0.5, y + 0.5, z + 0.5};
                if (dot3(r, normal) / len - dist < 0.0) solid[node_index(L, x, y, z)] = (unsigned char)id;
            }
}

/* ------------------------------------------------------------------------- */
/* Coupled system                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nv, nt, ne;
    int* tri;
    int* edge;
    int* hinge;
    int* hinge_tri;
    double *L0, *theta0, *S0, *hbar;
    double Sg0, V0;
    double k[5];
    int linear;
    int model;
} orc_tmpl;

struct orc_system {
    orc_lattice L;
    int n_tmpl, n_obj;
    orc_tmpl* t;
    int* o_tmpl;
    int* o_off;
    double* o_mass;
    double* o_fext;
    long M;
    double* Fel; /* [M][3] */
    double* Fprev; /* [M][3] total force of the last step (velocity Verlet) */
    int integrator;
    double* Frep; /* [M][3] soft-sphere forces of the current step */
    int* o_type;
    int n_pair, n_wall, n_shape;
    orc_soft_sphere* pair;
    orc_soft_sphere* wall;
    orc_shape* shape;
    double* G;   /* [3][N] */
    double* u;   /* [3][N] */
    double* rho; /* [N] */
    double* ntmp;
};

void orc_system_destroy(orc_system* s) {
    if (!s) return;
    for (int t = 0; t < s->n_tmpl; ++t) {
        free(s->t[t].tri);
        free(s->t[t].edge);
        free(s->t[t].hinge);
        free(s->t[t].hinge_tri);
        free(s->t[t].L0);
        free(s->t[t].theta0);
        free(s->t[t].S0);
        free(s->t[t].hbar);
    }
    free(s->t);
    free(s->o_tmpl);
    free(s->o_off);
    free(s->o_mass);
    free(s->o_fext);
    free(s->Fel);
    free(s->Fprev);
    free(s->Frep);
    free(s->o_type);
    free(s->pair);
    free(s->wall);
    free(s->shape);
    free(s->G);
    free(s->u);
    free(s->rho);
    free(s->ntmp);
    free(s);
}

orc_system* orc_system_create(const orc_lattice* L, const orc_mesh* m, const int* t_node_off,
                              const double* t_x) {
    orc_system* s = (orc_system*)calloc(1, sizeof(orc_system));
    s->L = *L;
    s->n_tmpl = m->n_tmpl;
    s->n_obj = m->n_obj;
    s->t = (orc_tmpl*)calloc((size_t)(m->n_tmpl > 0 ? m->n_tmpl : 1), sizeof(orc_tmpl));
    for (int t = 0; t < m->n_tmpl; ++t) {
        orc_tmpl* T = &s->t[t];
        T->nv = m->t_nv[t];
        T->nt = m->t_nt[t];
        int ne_max = 3 * T->nt / 2 + 1;
        T->tri = (int*)malloc(sizeof(int) * 3 * (size_t)T->nt);
        memcpy(T->tri, &m->tri[3 * (size_t)m->t_tri_off[t]], sizeof(int) * 3 * (size_t)T->nt);
        T->edge = (int*)malloc(sizeof(int) * 2 * (size_t)ne_max);
        T->hinge = (int*)malloc(sizeof(int) * 4 * (size_t)ne_max);
        T->hinge_tri = (int*)malloc(sizeof(int) * 2 * (size_t)ne_max);
        T->ne = orc_topology(T->nv, T->nt, T->tri, T->edge, T->hinge, T->hinge_tri);
        if (T->ne < 0) {
            orc_system_destroy(s);
            return NULL;
        }
        T->L0 = (double*)malloc(sizeof(double) * (size_t)T->ne);
        T->theta0 = (double*)malloc(sizeof(double) * (size_t)T->ne);
        T->S0 = (double*)malloc(sizeof(double) * (size_t)T->nt);
        orc_relaxed(T->nv, &t_x[3 * (size_t)t_node_off[t]], T->nt, T->tri, T->ne, T->edge,
                    T->hinge, T->L0, T->theta0, T->S0, &T->Sg0, &T->V0);
        T->hbar = (double*)malloc(sizeof(double) * (size_t)T->ne);
        orc_wing_height(T->nv, &t_x[3 * (size_t)t_node_off[t]], T->ne, T->hinge, T->hbar);
        for (int c = 0; c < 5; ++c) T->k[c] = m->t_k[5 * t + c];
        T->linear = m->t_linear[t];
        T->model = m->t_model ? m->t_model[t] : ORC_MODEL_PAPER;
    }
    s->o_tmpl = (int*)malloc(sizeof(int) * (size_t)(m->n_obj + 1));
    s->o_off = (int*)malloc(sizeof(int) * (size_t)(m->n_obj + 1));
    s->o_mass = (double*)malloc(sizeof(double) * (size_t)(m->n_obj + 1));
    s->o_fext = (double*)malloc(sizeof(double) * 3 * (size_t)(m->n_obj + 1));
    s->M = 0;
    for (int o = 0; o < m->n_obj; ++o) {
        s->o_tmpl[o] = m->o_tmpl[o];
        s->o_off[o] = m->o_node_off[o];
        s->o_mass[o] = m->o_mass[o];
        for (int c = 0; c < 3; ++c) s->o_fext[3 * o + c] = m->o_fext[3 * o + c];
        long end = (long)m->o_node_off[o] + s->t[m->o_tmpl[o]].nv;
        if (end > s->M) s->M = end;
    }
    long N = (long)L->nx * L->ny * L->nz;
    s->Fel = (double*)calloc((size_t)(3 * s->M + 1), sizeof(double));
    s->Fprev = (double*)calloc((size_t)(3 * s->M + 1), sizeof(double));
    s->integrator = m->integrator;
    s->Frep = (double*)calloc((size_t)(3 * s->M + 1), sizeof(double));
    s->o_type = (int*)calloc((size_t)(m->n_obj + 1), sizeof(int));
    for (int o = 0; o < m->n_obj; ++o) s->o_type[o] = m->o_type ? m->o_type[o] : 0;
    s->n_pair = m->n_pair;
    s->n_wall = m->n_wall;
    s->n_shape = m->n_shape;
    s->pair = (orc_soft_sphere*)calloc((size_t)(m->n_pair + 1), sizeof(orc_soft_sphere));
    s->wall = (orc_soft_sphere*)calloc((size_t)(m->n_wall + 1), sizeof(orc_soft_sphere));
    s->shape = (orc_shape*)calloc((size_t)(m->n_shape + 1), sizeof(orc_shape));
    if (m->n_pair) memcpy(s->pair, m->pair, sizeof(orc_soft_sphere) * (size_t)m->n_pair);
    if (m->n_wall) memcpy(s->wall, m->wall, sizeof(orc_soft_sphere) * (size_t)m->n_wall);
    if (m->n_shape) memcpy(s->shape, m->shape, sizeof(orc_shape) * (size_t)m->n_shape);
    s->G = (double*)calloc((size_t)(3 * N), sizeof(double));
    s->u = (double*)calloc((size_t)(3 * N), sizeof(double));
    s->rho = (double*)calloc((size_t)N, sizeof(double));
    s->ntmp = (double*)calloc((size_t)(19 * N), sizeof(double));
    return s;
}

void orc_system_geometry(orc_system* s, const double* X, double* Sg, double* Vol) {
    for (int o = 0; o < s->n_obj; ++o) {
        orc_tmpl* T = &s->t[s->o_tmpl[o]];
        orc_geometry(T->nv, &X[3 * (size_t)s->o_off[o]], T->nt, T->tri, NULL, &Sg[o], &Vol[o]);
    }
}

void orc_system_forces(orc_system* s, const double* X, double* F) {
    memset(F, 0, sizeof(double) * 3 * (size_t)s->M);
    for (int o = 0; o < s->n_obj; ++o) {
        orc_tmpl* T = &s->t[s->o_tmpl[o]];
        size_t off = 3 * (size_t)s->o_off[o];
        orc_membrane_forces(T->nv, &X[off], T->nt, T->tri, T->ne, T->edge, T->hinge, T->L0,
                            T->theta0, T->S0, T->Sg0, T->V0, T->k, T->linear, T->model, T->hbar,
                            &F[off]);
    }
}

/* ------------------------------------------------------------------------- */
/* Soft-sphere repulsion (the collisions the paper's scripts switch on)       */
/* ------------------------------------------------------------------------- */
static void soft_sphere_force(const orc_soft_sphere* ss, double d, const double* dir, double* F) {
    /* force a n (d - offset)^-(n+1) along dir inside the interaction range */
    double e = d - ss->offset;
    if (!(e > 0.0 && e < ss->cutoff)) return;
    double f = ss->a * ss->n * pow(e, -(ss->n + 1.0));
    for (int c = 0; c < 3; ++c) F[c] += f * dir[c];
}

static void consider(const double* x, const double* p, double* best, double* bp) {
    double r[3];
    sub3(x, p, r);
    double d = norm3(r);
    if (d < *best) {
        *best = d;
        for (int c = 0; c < 3; ++c) bp[c] = p[c];
    }
}

int orc_shape_distance(const orc_shape* sh, const double* x, double* dist, double* dir) {
    if (sh->kind == 1) {  /* half-space n.x < dist is solid */
        double len = norm3(sh->normal);
        double d = dot3(x, sh->normal) / len - sh->dist;
        if (!(d > 0.0)) return 0;
        *dist = d;
        for (int c = 0; c < 3; ++c) dir[c] = sh->normal[c] / len;
        return 1;
    }
    /* rhomboid: inside when all three Cramer coordinates lie in [0, 1] */
    const double* E[3] = {sh->a, sh->b, sh->c};
    double r[3], bc[3], ca[3], ab[3];
    sub3(x, sh->corner, r);
    cross3(sh->b, sh->c, bc);
    cross3(sh->c, sh->a, ca);
    cross3(sh->a, sh->b, ab);
    double det = dot3(sh->a, bc);
    double st[3] = {dot3(r, bc) / det, dot3(r, ca) / det, dot3(r, ab) / det};
    if (st[0] >= 0.0 && st[0] <= 1.0 && st[1] >= 0.0 && st[1] <= 1.0 && st[2] >= 0.0 && st[2] <= 1.0)
        return 0;
    /* closest surface point: the best of the face interiors, the edges and the
     * corners (the closest point of a convex body is one of them) */
    double best = INFINITY, bp[3] = {0, 0, 0}, p[3];
    for (int k = 0; k < 3; ++k) {          /* faces with coordinate k fixed */
        const double* u = E[(k + 1) % 3];
        const double* v = E[(k + 2) % 3];
        for (int side = 0; side < 2; ++side) {
            double o[3], q[3];
            for (int c = 0; c < 3; ++c) o[c] = sh->corner[c] + side * E[k][c];
            sub3(x, o, q);
            double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v);
            double qu = dot3(q, u), qv = dot3(q, v);
            double den = uu * vv - uv * uv;
            double su = (qu * vv - qv * uv) / den, sv = (qv * uu - qu * uv) / den;
            if (su >= 0.0 && su <= 1.0 && sv >= 0.0 && sv <= 1.0) {
                for (int c = 0; c < 3; ++c) p[c] = o[c] + su * u[c] + sv * v[c];
                consider(x, p, &best, bp);
            }
        }
    }
    for (int k = 0; k < 3; ++k)            /* edges along E[k] */
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const double* u = E[(k + 1) % 3];
                const double* v = E[(k + 2) % 3];
                double o[3], q[3];
                for (int c = 0; c < 3; ++c) o[c] = sh->corner[c] + i * u[c] + j * v[c];
                sub3(x, o, q);
                double t = dot3(q, E[k]) / dot3(E[k], E[k]);
                t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                for (int c = 0; c < 3; ++c) p[c] = o[c] + t * E[k][c];
                consider(x, p, &best, bp);
            }
    *dist = best;
    double rr[3];
    sub3(x, bp, rr);
    for (int c = 0; c < 3; ++c) dir[c] = rr[c] / best;
    return 1;
}

/* the interaction of two types: the last entry that names them */
static const orc_soft_sphere* pair_of(const orc_system* s, int ta, int tb) {
    const orc_soft_sphere* r = NULL;
    for (int k = 0; k < s->n_pair; ++k)
        if ((s->pair[k].type_a == ta && s->pair[k].type_b == tb) ||
            (s->pair[k].type_a == tb && s->pair[k].type_b == ta))
            r = &s->pair[k];
    return r;
}

void orc_system_repulsion(orc_system* s, const double* X, double* F) {
    const orc_lattice* L = &s->L;
    double box[3] = {L->nx, L->ny, L->nz};
    int periodic[3] = {1, 1, !L->walls_z};
    /* node pairs (each unordered pair once) */
    for (int o1 = 0; o1 < s->n_obj; ++o1)
        for (int o2 = o1; o2 < s->n_obj; ++o2) {
            const orc_soft_sphere* ss = pair_of(s, s->o_type[o1], s->o_type[o2]);
            if (!ss) continue;
            int n1 = s->t[s->o_tmpl[o1]].nv, n2 = s->t[s->o_tmpl[o2]].nv;
            for (int v1 = 0; v1 < n1; ++v1)
                for (int v2 = (o1 == o2 ? v1 + 1 : 0); v2 < n2; ++v2) {
                    long j = (long)s->o_off[o1] + v1, k = (long)s->o_off[o2] + v2;
                    double r[3];
                    for (int c = 0; c < 3; ++c) {
                        r[c] = X[3 * j + c] - X[3 * k + c];
                        if (periodic[c]) r[c] -= box[c] * floor(r[c] / box[c] + 0.5);
                    }
                    double d = norm3(r);
                    if (!(d > ss->offset && d < ss->offset + ss->cutoff)) continue;
                    double dir[3] = {r[0] / d, r[1] / d, r[2] / d}, f[3] = {0, 0, 0};
                    soft_sphere_force(ss, d, dir, f);
                    for (int c = 0; c < 3; ++c) {
                        F[3 * j + c] += f[c];
                        F[3 * k + c] -= f[c];
                    }
                }
        }
    /* walls: every obstacle shape at the node's position in the box, and the
     * built-in walls z = 0 and z = nz */
    for (int o = 0; o < s->n_obj; ++o) {
        const orc_soft_sphere* ss = NULL;
        for (int k = 0; k < s->n_wall; ++k)
            if (s->wall[k].type_a == s->o_type[o]) ss = &s->wall[k];
        if (!ss) continue;
        int nv = s->t[s->o_tmpl[o]].nv;
        for (int v = 0; v < nv; ++v) {
            long j = (long)s->o_off[o] + v;
            double x[3];
            for (int c = 0; c < 3; ++c) {
                x[c] = X[3 * j + c];
                if (periodic[c]) x[c] -= box[c] * floor(x[c] / box[c]);
            }
            for (int k = 0; k < s->n_shape; ++k) {
                double d, dir[3];
                if (orc_shape_distance(&s->shape[k], x, &d, dir)) soft_sphere_force(ss, d, dir, &F[3 * j]);
            }
            if (L->walls_z) {
                double up[3] = {0, 0, 1}, down[3] = {0, 0, -1};
                if (x[2] > 0.0) soft_sphere_force(ss, x[2], up, &F[3 * j]);
                if (x[2] < L->nz) soft_sphere_force(ss, L->nz - x[2], down, &F[3 * j]);
            }
        }
    }
}

long orc_system_touched(orc_system* s, const double* X) {
    long N = (long)s->L.nx * s->L.ny * s->L.nz;
    unsigned char* mark = (unsigned char*)calloc((size_t)N, 1);
    long cnt = 0;
    for (long j = 0; j < s->M; ++j) {
        long idx[8];
        double w[8];
        orc_stencil(&s->L, &X[3 * j], idx, w);
        for (int k = 0; k < 8; ++k)
            if (!mark[idx[k]]) {
                mark[idx[k]] = 1;
                ++cnt;
            }
    }
    free(mark);
    return cnt;
}

void orc_system_get_force(const orc_system* s, double* F) {
    memcpy(F, s->Fprev, sizeof(double) * 3 * (size_t)s->M);
}

void orc_system_set_force(orc_system* s, const double* F) {
    memcpy(s->Fprev, F, sizeof(double) * 3 * (size_t)s->M);
}

int orc_system_run(orc_system* s, double* n, double* X, double* V, int n_steps, double* diag) {
    const orc_lattice* L = &s->L;
    long N = (long)L->nx * L->ny * L->nz;
    int verlet = s->integrator == ORC_VERLET;
    int repulsion = s->n_pair > 0 || s->n_wall > 0;
    for (int step = 0; step < n_steps; ++step) {
        double d[13] = {0};
        /* a non-finite mesh state has no stencil: stop instead of indexing */
        for (long j = 0; j < 3 * s->M; ++j)
            if (!isfinite(X[j]) || !isfinite(V[j]) || fabs(X[j]) > 1e9) return -1 - step;
        if (verlet) {
            /* velocity Verlet, first half: half kick with the force of the
             * previous step, then drift; V holds the half-step velocity */
            for (int o = 0; o < s->n_obj; ++o) {
                int nv = s->t[s->o_tmpl[o]].nv;
                double m = s->o_mass[o];
                for (int v = 0; v < nv; ++v) {
                    long j = (long)s->o_off[o] + v;
                    for (int c = 0; c < 3; ++c) {
                        V[3 * j + c] += 0.5 * s->Fprev[3 * j + c] / m;
                        X[3 * j + c] += V[3 * j + c];
                    }
                }
            }
        }
        /* 1-2: geometry and membrane forces from the current positions (step
         * start; after the drift with velocity Verlet) */
        orc_system_forces(s, X, s->Fel);
        memset(s->Frep, 0, sizeof(double) * 3 * (size_t)s->M);
        if (repulsion) orc_system_repulsion(s, X, s->Frep);
        /* 3: coupling.  Node velocity from the populations at step start,
         * with half the body force only. */
        orc_moments(L, n, NULL, s->rho, s->u);
        memset(s->G, 0, sizeof(double) * 3 * (size_t)N);
        for (int o = 0; o < s->n_obj; ++o) {
            int nv = s->t[s->o_tmpl[o]].nv;
            double m = s->o_mass[o];
            for (int v = 0; v < nv; ++v) {
                long j = (long)s->o_off[o] + v;
                double drag[3]; /* xi (v - u): the force handed to the fluid */
                d[0] += orc_couple_point(L, s->u, &X[3 * j], &V[3 * j], s->G, drag);
                /* 4: mesh update: kick then drift (Euler) or the second half
                 * kick (velocity Verlet) */
                for (int c = 0; c < 3; ++c) {
                    double Ft = s->Fel[3 * j + c] - drag[c] + s->o_fext[3 * o + c] + s->Frep[3 * j + c];
                    if (verlet) {
                        V[3 * j + c] += 0.5 * Ft / m;
                        s->Fprev[3 * j + c] = Ft;
                    } else {
                        V[3 * j + c] += Ft / m;
                        X[3 * j + c] += V[3 * j + c];
                    }
                    d[1 + c] += s->Fel[3 * j + c];
                    d[4 + c] += -drag[c];
                    d[7 + c] += s->o_fext[3 * o + c];
                    d[10 + c] += s->Frep[3 * j + c];
                }
            }
        }
        /* 5: lattice Boltzmann update with force density g + G */
        orc_lb_step(L, n, s->G, s->ntmp);
        memcpy(n, s->ntmp, sizeof(double) * 19 * (size_t)N);
        if (diag && step == n_steps - 1) memcpy(diag, d, sizeof(d));
    }
    return 0;
}
