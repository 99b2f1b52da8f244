/*
 * FP64 CPU oracle of the DSDP docking stage (arXiv 2303.09916).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct double-precision code
 * that the test-suite, the smoke check and the benchmark's CPU-baseline leg use to
 * judge the GPU library.  The product path never links, loads or calls it, and it
 * shares no code, header, table or helper with the GPU library.
 *
 * What it follows:
 *   - Vina scoring, kept unchanged by the paper (Section 2, "Binding pose search",
 *     opening paragraph; ref. [6], Trott & Olson 2010): five terms on the surface
 *     distance d = r - R_a - R_b with an 8 A cutoff on r.  The paper prints none of
 *     the terms or weights; the published Vina values are used.
 *   - Grid maps (Section 2, first modification; Appendix eq. 1): each node holds the
 *     summed interaction of one ligand atom type with every receptor atom within the
 *     cutoff, and the gradient of that sum (the score-and-gradient grids).
 *   - Trilinear interpolation (Appendix eq. 2) of the energy and of the stored
 *     gradient (Appendix eq. 4).  The derivative of the interpolated energy
 *     (Appendix eq. 3) is available as a reference mode only.
 *   - Local optimisation: BFGS (Section 2, second modification names Vina's BFGS,
 *     ref. [36]); Armijo backtracking line search.
 *   - Monte Carlo with many short independent chains (Section 2, parallelisation
 *     paragraph); CPU post-processing of the chain results into ranked poses
 *     (same paragraph; Figure 4), heavy-atom RMSD (Section 2, "Baseline Setup").
 *
 * Everything the paper leaves open (ligand model, move set, constants, wall,
 * ranking) is a stated reading, documented next to the code that implements it.
 *
 * Parity pins: every function here is checked by tests against closed forms,
 * brute force, finite differences, invariants or published test vectors.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NXS 17
#define ORC_CUTOFF 8.0
#define ORC_MAX_ATOMS 64
#define ORC_MAX_FRAGS 32
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* XS atom types (Vina ref. [6]): radius, hydrophobic, donor, acceptor.       */
/* Order: C_H C_P N_P N_D N_A N_DA O_P O_D O_A O_DA S_P P_P F_H Cl_H Br_H I_H Met_D */
/* ------------------------------------------------------------------------- */
static const double XS_RADIUS[ORC_NXS] = {
    1.9, 1.9, 1.8, 1.8, 1.8, 1.8, 1.7, 1.7, 1.7, 1.7, 2.0, 2.1, 1.5, 1.8, 2.0, 2.2, 1.2};
static const int XS_HYDROPHOBIC[ORC_NXS] = {1,0,0,0,0,0,0,0,0,0,0,0,1,1,1,1,0};
static const int XS_DONOR[ORC_NXS]       = {0,0,0,1,0,1,0,1,0,1,0,0,0,0,0,0,1};
static const int XS_ACCEPTOR[ORC_NXS]    = {0,0,0,0,1,1,0,0,1,1,0,0,0,0,0,0,0};

/* Vina weights (ref. [6]): gauss1, gauss2, repulsion, hydrophobic, hydrogen bond. */
static const double W_GAUSS1 = -0.0356;
static const double W_GAUSS2 = -0.00516;
static const double W_REPULSION = 0.840;
static const double W_HYDROPHOBIC = -0.0351;
static const double W_HBOND = -0.587;
/* Vina's rotatable-bond normalisation of the final score. */
static const double W_ROT = 0.0585;

int orc_n_xs(void) { return ORC_NXS; }

/*
 * Unweighted Vina terms of one atom pair at centre distance r (ref. [6]):
 *   gauss1 = exp(-(d/0.5)^2); gauss2 = exp(-((d-3)/2)^2); repulsion = d^2 for d<0;
 *   hydrophobic: 1 below d=0.5, 0 above d=1.5, linear between (hydrophobic pairs);
 *   hbond: 1 below d=-0.7, 0 above d=0, linear between (donor-acceptor pairs).
 * All terms vanish for r >= 8 (hard cutoff).  dterms (nullable) receives the
 * derivatives with respect to d; at a kink the left-hand derivative is taken.
 * Returns the weighted sum.
 */
double orc_pair_terms(int ta, int tb, double r, double *terms, double *dterms)
{
    double t[5] = {0, 0, 0, 0, 0}, dt[5] = {0, 0, 0, 0, 0};
    if (r < ORC_CUTOFF) {
        double d = r - XS_RADIUS[ta] - XS_RADIUS[tb];
        double a = d / 0.5;
        t[0] = exp(-a * a);
        dt[0] = t[0] * (-2.0 * a / 0.5);
        double b = (d - 3.0) / 2.0;
        t[1] = exp(-b * b);
        dt[1] = t[1] * (-2.0 * b / 2.0);
        if (d < 0.0) { t[2] = d * d; dt[2] = 2.0 * d; }
        if (XS_HYDROPHOBIC[ta] && XS_HYDROPHOBIC[tb]) {
            if (d <= 0.5) { t[3] = 1.0; dt[3] = 0.0; }
            else if (d <= 1.5) { t[3] = 1.5 - d; dt[3] = -1.0; }
        }
        if ((XS_DONOR[ta] && XS_ACCEPTOR[tb]) || (XS_DONOR[tb] && XS_ACCEPTOR[ta])) {
            if (d <= -0.7) { t[4] = 1.0; dt[4] = 0.0; }
            else if (d <= 0.0) { t[4] = -d / 0.7; dt[4] = -1.0 / 0.7; }
        }
    }
    if (terms) memcpy(terms, t, sizeof t);
    if (dterms) memcpy(dterms, dt, sizeof dt);
    return W_GAUSS1 * t[0] + W_GAUSS2 * t[1] + W_REPULSION * t[2] + W_HYDROPHOBIC * t[3] + W_HBOND * t[4];
}

/* Weighted pair energy h_ab(r) and dh/dr (= dh/dd). */
double orc_pair_energy(int ta, int tb, double r, double *dedr)
{
    double t[5], dt[5];
    double e = orc_pair_terms(ta, tb, r, t, dt);
    if (dedr)
        *dedr = W_GAUSS1 * dt[0] + W_GAUSS2 * dt[1] + W_REPULSION * dt[2] + W_HYDROPHOBIC * dt[3] + W_HBOND * dt[4];
    return e;
}

/* Sum of the absolute weighted terms, and of absolute weighted derivatives. */
static void pair_mass(int ta, int tb, double r, double *me, double *mg)
{
    double t[5], dt[5];
    orc_pair_terms(ta, tb, r, t, dt);
    const double w[5] = {W_GAUSS1, W_GAUSS2, W_REPULSION, W_HYDROPHOBIC, W_HBOND};
    double a = 0, b = 0;
    for (int k = 0; k < 5; k++) { a += fabs(w[k] * t[k]); b += fabs(w[k] * dt[k]); }
    *me = a; *mg = b;
}

/*
 * Near-tie mass of one pair: the energy or derivative that a rounding-level change
 * of r could switch on or off.  Within eps of the cutoff the whole term can
 * appear or vanish; within eps of a kink of the piecewise-linear terms the
 * derivative can take either branch.
 */
static void pair_tie(int ta, int tb, double r, double eps, double *te, double *tg)
{
    *te = 0; *tg = 0;
    if (fabs(r - ORC_CUTOFF) < eps) {
        double dd;
        double e = orc_pair_energy(ta, tb, ORC_CUTOFF - eps, &dd);
        *te += fabs(e);
        *tg += fabs(dd);
    }
    if (r >= ORC_CUTOFF + eps) return;
    double d = r - XS_RADIUS[ta] - XS_RADIUS[tb];
    if (XS_HYDROPHOBIC[ta] && XS_HYDROPHOBIC[tb])
        if (fabs(d - 0.5) < eps || fabs(d - 1.5) < eps) *tg += fabs(W_HYDROPHOBIC);
    if ((XS_DONOR[ta] && XS_ACCEPTOR[tb]) || (XS_DONOR[tb] && XS_ACCEPTOR[ta]))
        if (fabs(d + 0.7) < eps || fabs(d) < eps) *tg += fabs(W_HBOND) / 0.7;
}

/* ------------------------------------------------------------------------- */
/* Grid geometry and maps (Appendix eq. 1; Section 2, first modification).    */
/* ------------------------------------------------------------------------- */

/* n = floor(size/h) + 1 nodes per axis, centred on the box centre. */
void orc_grid_geometry(const double *centre, const double *size, double h, int *n, double *origin)
{
    for (int a = 0; a < 3; a++) {
        n[a] = (int)floor(size[a] / h) + 1;
        origin[a] = centre[a] - 0.5 * (n[a] - 1) * h;
    }
}

/*
 * Value and gradient of map type t at point m by direct summation over all
 * receptor atoms (eq. 1 and its gradient):
 *   E = sum_j h(t, type_j, |m - r_j|),  G = sum_j h'(d) (m - r_j)/|m - r_j|.
 * A pair at r < 1e-9 contributes to E but not to G (the direction is undefined).
 * out[0..3] = E, Gx, Gy, Gz; mass (nullable) = {sum |terms|, sum |h'|};
 * tie (nullable) = {energy tie mass, gradient tie mass}.
 */
static void direct_point(const double *rec, const int *rtype, int n_rec, int t, const double *m,
                         double *out, double *mass, double *tie, double tie_eps)
{
    double E = 0, G[3] = {0, 0, 0}, me = 0, mg = 0, te = 0, tg = 0;
    for (int j = 0; j < n_rec; j++) {
        double dx = m[0] - rec[3 * j], dy = m[1] - rec[3 * j + 1], dz = m[2] - rec[3 * j + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (tie) {
            double a, b;
            pair_tie(t, rtype[j], r, tie_eps, &a, &b);
            te += a; tg += b;
        }
        if (r >= ORC_CUTOFF) continue;
        double dd;
        E += orc_pair_energy(t, rtype[j], r, &dd);
        if (r > 1e-9) { G[0] += dd * dx / r; G[1] += dd * dy / r; G[2] += dd * dz / r; }
        if (mass) { double a, b; pair_mass(t, rtype[j], r, &a, &b); me += a; mg += b; }
    }
    out[0] = E; out[1] = G[0]; out[2] = G[1]; out[3] = G[2];
    if (mass) { mass[0] = me; mass[1] = mg; }
    if (tie) { tie[0] = te; tie[1] = tg; }
}

/*
 * Full maps, layout maps[t][k][j][i][4] with node (i,j,k) at origin + h*(i,j,k).
 * use_cells = 0: every receptor atom is visited for every node (brute force).
 * use_cells = 1: receptor atoms are binned into cubic cells of edge `cell` and
 * only cells within the cutoff are visited; the pair sum is the same set of
 * terms, so the result equals brute force up to summation order.
 * mass and tie are nullable, layout [t][k][j][i][2].
 */
void orc_build_grid(const float *rec_xyz, const int *rec_type, int n_rec, const double *origin, const int *n,
                    double h, const int *map_types, int T, int use_cells, double cell,
                    double *maps, double *mass, double *tie, double tie_eps)
{
    double *rec = (double *)malloc(sizeof(double) * 3 * (n_rec > 0 ? n_rec : 1));
    for (int j = 0; j < 3 * n_rec; j++) rec[j] = (double)rec_xyz[j];
    const long nodes = (long)n[0] * n[1] * n[2];

    /* cell binning (counting sort by cell key) */
    int cn[3] = {1, 1, 1};
    double clo[3] = {0, 0, 0};
    int *cstart = NULL, *corder = NULL;
    if (use_cells && n_rec > 0) {
        double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
        for (int j = 0; j < n_rec; j++)
            for (int a = 0; a < 3; a++) {
                if (rec[3 * j + a] < lo[a]) lo[a] = rec[3 * j + a];
                if (rec[3 * j + a] > hi[a]) hi[a] = rec[3 * j + a];
            }
        for (int a = 0; a < 3; a++) { clo[a] = lo[a]; cn[a] = (int)floor((hi[a] - lo[a]) / cell) + 1; }
        long ncell = (long)cn[0] * cn[1] * cn[2];
        cstart = (int *)calloc(ncell + 1, sizeof(int));
        corder = (int *)malloc(sizeof(int) * n_rec);
        int *key = (int *)malloc(sizeof(int) * n_rec);
        for (int j = 0; j < n_rec; j++) {
            int c[3];
            for (int a = 0; a < 3; a++) {
                c[a] = (int)floor((rec[3 * j + a] - clo[a]) / cell);
                if (c[a] < 0) c[a] = 0;
                if (c[a] >= cn[a]) c[a] = cn[a] - 1;
            }
            key[j] = (c[2] * cn[1] + c[1]) * cn[0] + c[0];
            cstart[key[j] + 1]++;
        }
        for (long c = 0; c < ncell; c++) cstart[c + 1] += cstart[c];
        int *fill = (int *)malloc(sizeof(int) * ncell);
        for (long c = 0; c < ncell; c++) fill[c] = cstart[c];
        for (int j = 0; j < n_rec; j++) corder[fill[key[j]]++] = j;
        free(fill);
        free(key);
    }
    const int reach = use_cells ? (int)ceil(ORC_CUTOFF / cell) : 0;

#pragma omp parallel for schedule(dynamic, 64)
    for (long node = 0; node < nodes; node++) {
        int i = (int)(node % n[0]);
        int jy = (int)((node / n[0]) % n[1]);
        int k = (int)(node / ((long)n[0] * n[1]));
        double m[3] = {origin[0] + h * i, origin[1] + h * jy, origin[2] + h * k};
        for (int t = 0; t < T; t++) {
            int tt = map_types[t];
            double out[4], ms[2], ti[2];
            if (!use_cells) {
                direct_point(rec, rec_type, n_rec, tt, m, out, ms, ti, tie_eps);
            } else {
                double E = 0, G[3] = {0, 0, 0}, me = 0, mg = 0, te = 0, tg = 0;
                int c0[3];
                for (int a = 0; a < 3; a++) c0[a] = (int)floor((m[a] - clo[a]) / cell);
                for (int cz = c0[2] - reach; cz <= c0[2] + reach; cz++) {
                    if (cz < 0 || cz >= cn[2]) continue;
                    for (int cy = c0[1] - reach; cy <= c0[1] + reach; cy++) {
                        if (cy < 0 || cy >= cn[1]) continue;
                        for (int cx = c0[0] - reach; cx <= c0[0] + reach; cx++) {
                            if (cx < 0 || cx >= cn[0]) continue;
                            long c = ((long)cz * cn[1] + cy) * cn[0] + cx;
                            for (int q = cstart[c]; q < cstart[c + 1]; q++) {
                                int j = corder[q];
                                double dx = m[0] - rec[3 * j], dy = m[1] - rec[3 * j + 1], dz = m[2] - rec[3 * j + 2];
                                double r = sqrt(dx * dx + dy * dy + dz * dz);
                                double a, b;
                                pair_tie(tt, rec_type[j], r, tie_eps, &a, &b);
                                te += a; tg += b;
                                if (r >= ORC_CUTOFF) continue;
                                double dd;
                                E += orc_pair_energy(tt, rec_type[j], r, &dd);
                                if (r > 1e-9) { G[0] += dd * dx / r; G[1] += dd * dy / r; G[2] += dd * dz / r; }
                                pair_mass(tt, rec_type[j], r, &a, &b);
                                me += a; mg += b;
                            }
                        }
                    }
                }
                out[0] = E; out[1] = G[0]; out[2] = G[1]; out[3] = G[2];
                ms[0] = me; ms[1] = mg; ti[0] = te; ti[1] = tg;
            }
            long base = (long)t * nodes + node;
            for (int c = 0; c < 4; c++) maps[4 * base + c] = out[c];
            if (mass) { mass[2 * base] = ms[0]; mass[2 * base + 1] = ms[1]; }
            if (tie) { tie[2 * base] = ti[0]; tie[2 * base + 1] = ti[1]; }
        }
    }
    free(rec);
    free(cstart);
    free(corder);
}

/*
 * Map values at a list of sampled nodes, by direct summation (for checking large
 * grids one node at a time).  sel[s] = linear index t*nodes + node.
 */
void orc_grid_nodes(const float *rec_xyz, const int *rec_type, int n_rec, const double *origin, const int *n,
                    double h, const int *map_types, const long *sel, int n_sel,
                    double *out, double *mass, double *tie, double tie_eps)
{
    double *rec = (double *)malloc(sizeof(double) * 3 * (n_rec > 0 ? n_rec : 1));
    for (int j = 0; j < 3 * n_rec; j++) rec[j] = (double)rec_xyz[j];
    const long nodes = (long)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(dynamic, 16)
    for (int s = 0; s < n_sel; s++) {
        long t = sel[s] / nodes, node = sel[s] % nodes;
        int i = (int)(node % n[0]);
        int jy = (int)((node / n[0]) % n[1]);
        int k = (int)(node / ((long)n[0] * n[1]));
        double m[3] = {origin[0] + h * i, origin[1] + h * jy, origin[2] + h * k};
        direct_point(rec, rec_type, n_rec, map_types[t], m, out + 4 * s, mass ? mass + 2 * s : NULL,
                     tie ? tie + 2 * s : NULL, tie_eps);
    }
    free(rec);
}

/* ------------------------------------------------------------------------- */
/* Trilinear interpolation (Appendix eqs. 2, 3, 4) with the box wall.         */
/* ------------------------------------------------------------------------- */

typedef struct {
    const double *maps;   /* [T][nz][ny][nx][4] */
    const double *mass;   /* nullable [T][nz][ny][nx][2] */
    const double *tie;    /* nullable [T][nz][ny][nx][2] */
    int n[3];
    double origin[3];
    double h;
    int T;
    int map_of_type[ORC_NXS];
    /* adaptive search space (Section 2, third modification): the box intersected
       with the union of balls of radius site_r around the site points */
    int n_site;
    double *site;         /* [n_site][3] */
    double site_r;
} orc_grid;

orc_grid *orc_grid_create(const double *maps, const double *mass, const double *tie, const int *n,
                          const double *origin, double h, const int *map_types, int T)
{
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    g->maps = maps; g->mass = mass; g->tie = tie;
    for (int a = 0; a < 3; a++) { g->n[a] = n[a]; g->origin[a] = origin[a]; }
    g->h = h; g->T = T;
    for (int x = 0; x < ORC_NXS; x++) g->map_of_type[x] = -1;
    for (int t = 0; t < T; t++) g->map_of_type[map_types[t]] = t;
    return g;
}

void orc_grid_free(orc_grid *g)
{
    if (g) free(g->site);
    free(g);
}

/* Site points of the adaptive search space; n = 0 restores the plain box. */
void orc_grid_set_site(orc_grid *g, const double *pts, int n, double radius)
{
    free(g->site);
    g->site = NULL;
    g->n_site = 0;
    if (n <= 0) return;
    g->site = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(g->site, pts, sizeof(double) * 3 * (size_t)n);
    g->n_site = n;
    g->site_r = radius;
}

/*
 * Restraint of the ligand's root position p to the adaptive search space
 * (reading of Section 2, third modification, and Figure 3): with site points,
 * the nearest one c (lowest index on ties) at distance d; outside its ball
 * (d > r) the pose pays wall_slope * (d - r), with gradient
 * wall_slope * (p - c) / d on p.  Returns the energy; adds the gradient to g3.
 */
double orc_site_term(const orc_grid *g, const double *p, double wall_slope, double *g3)
{
    if (g->n_site <= 0) return 0.0;
    int m = 0;
    double best = DBL_MAX;
    for (int i = 0; i < g->n_site; i++) {
        double d2 = 0;
        for (int a = 0; a < 3; a++) d2 += (p[a] - g->site[3 * i + a]) * (p[a] - g->site[3 * i + a]);
        if (d2 < best) { best = d2; m = i; }
    }
    double d = sqrt(best);
    if (d <= g->site_r) return 0.0;
    if (g3)
        for (int a = 0; a < 3; a++) g3[a] += wall_slope * (p[a] - g->site[3 * m + a]) / d;
    return wall_slope * (d - g->site_r);
}

enum { ORC_MODE_EQ4 = 0, ORC_MODE_EQ3 = 1, ORC_MODE_DIRECT = 2 };

/*
 * Interpolated energy and gradient of map `t` at point x.
 *   Per axis the grid coordinate is u = (x - origin)/h.  A coordinate outside
 *   [0, n-1] is clamped onto the box face; the atom then pays the wall energy
 *   wall_slope * (distance outside, in A) and its gradient along that axis is the
 *   wall's outward slope (the map gradient along a clamped axis is dropped, since
 *   the clamped energy does not change along it).  This is our reading of the
 *   wall restraint that Section 3 calls for (site-prediction paragraph).
 *   Cell index i = min(floor(u), n-2), fraction p = u - i (a point on the upper
 *   face gets i = n-2, p = 1).  Corner weights are products of p and 1-p (eq. 2).
 *   mode EQ4: gradient = the same weights applied to the stored gradients (eq. 4).
 *   mode EQ3: gradient = exact derivative of the eq. 2 interpolant (eq. 3), with
 *   (2l-1)/l_x read as +-1/h.
 * wall_out receives the wall energy (included in *E).  mass/tie (nullable) get the
 * interpolated map masses plus wall contributions.
 */
static void interp(const orc_grid *g, int t, const double *x, int mode, double wall_slope,
                   double *E, double *grad, double *wall_out, double *mass, double *tie, double tie_eps)
{
    double u[3], p[3], wall = 0, wg[3] = {0, 0, 0};
    int idx[3], clamped[3];
    for (int a = 0; a < 3; a++) {
        double lo = g->origin[a], hi = g->origin[a] + (g->n[a] - 1) * g->h;
        double xa = x[a];
        clamped[a] = 0;
        if (xa < lo) { wall += wall_slope * (lo - xa); wg[a] = -wall_slope; xa = lo; clamped[a] = 1; }
        else if (xa > hi) { wall += wall_slope * (xa - hi); wg[a] = wall_slope; xa = hi; clamped[a] = 1; }
        u[a] = (xa - lo) / g->h;
        int i = (int)floor(u[a]);
        if (i > g->n[a] - 2) i = g->n[a] - 2;
        if (i < 0) i = 0;
        idx[a] = i;
        p[a] = u[a] - i;
    }
    const long nodes = (long)g->n[0] * g->n[1] * g->n[2];
    double e = 0, gr[3] = {0, 0, 0}, me = 0, mg = 0, te = 0, tg = 0;
    for (int l = 0; l < 2; l++)
        for (int m = 0; m < 2; m++)
            for (int nn = 0; nn < 2; nn++) {
                double wx = l ? p[0] : 1 - p[0];
                double wy = m ? p[1] : 1 - p[1];
                double wz = nn ? p[2] : 1 - p[2];
                long node = ((long)(idx[2] + nn) * g->n[1] + (idx[1] + m)) * g->n[0] + (idx[0] + l);
                long base = (long)t * nodes + node;
                const double *c = g->maps + 4 * base;
                double w = wx * wy * wz;
                e += w * c[0];
                if (mode == ORC_MODE_EQ4) {
                    gr[0] += w * c[1]; gr[1] += w * c[2]; gr[2] += w * c[3];
                } else {
                    double sx = (2 * l - 1) / g->h, sy = (2 * m - 1) / g->h, sz = (2 * nn - 1) / g->h;
                    gr[0] += sx * wy * wz * c[0];
                    gr[1] += wx * sy * wz * c[0];
                    gr[2] += wx * wy * sz * c[0];
                }
                if (g->mass) { me += w * g->mass[2 * base]; mg += w * g->mass[2 * base + 1]; }
                if (g->tie) { te += w * g->tie[2 * base]; tg += w * g->tie[2 * base + 1]; }
            }
    for (int a = 0; a < 3; a++) if (clamped[a]) gr[a] = 0;
    *E = e + wall;
    for (int a = 0; a < 3; a++) grad[a] = gr[a] + wg[a];
    *wall_out = wall;
    if (mass) { mass[0] = me + wall; mass[1] = mg + (wall > 0 ? wall_slope : 0); }
    if (tie) {
        double wt = 0;
        for (int a = 0; a < 3; a++) {
            double lo = g->origin[a], hi = g->origin[a] + (g->n[a] - 1) * g->h;
            if (fabs(x[a] - lo) < tie_eps || fabs(x[a] - hi) < tie_eps) wt += wall_slope + fabs(gr[a]) + 1.0;
        }
        tie[0] = te;
        tie[1] = tg + wt;
    }
}

void orc_interp(const orc_grid *g, int t, const double *x, int mode, double wall_slope, double *out)
{
    double w;
    interp(g, t, x, mode, wall_slope, &out[0], &out[1], &w, NULL, NULL, 0);
}

/* ------------------------------------------------------------------------- */
/* Ligand model: torsion tree and forward kinematics (Vina's model, ref. [6]). */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n_atoms, n_frags, n_tors;
    double ref[ORC_MAX_ATOMS][3];
    int type[ORC_MAX_ATOMS];
    int frag_of[ORC_MAX_ATOMS];
    int frag_start[ORC_MAX_FRAGS + 1];
    int parent[ORC_MAX_FRAGS];
    int axis_a[ORC_MAX_FRAGS], axis_b[ORC_MAX_FRAGS];
    double root_centre[3];
    double rg;                    /* gyration radius about the root centre */
    int n_pairs;
    int pair_i[ORC_MAX_ATOMS * ORC_MAX_ATOMS / 2], pair_j[ORC_MAX_ATOMS * ORC_MAX_ATOMS / 2];
    int in_subtree[ORC_MAX_FRAGS][ORC_MAX_FRAGS];   /* in_subtree[k][m]: m lies in the subtree of k */
} orc_ligand;

/*
 * Ligand from the library's description.  Atoms are fragment-contiguous;
 * fragment k >= 1 hangs off parent[k] < k and turns about the bond
 * (axis[2k] in the parent, axis[2k+1] in k).  Returns NULL on invalid input.
 *
 * Intra-ligand pairs (reading; the paper keeps Vina's scoring): pairs of atoms in
 * different fragments that are more than three bonds apart.  Pairs inside one
 * rigid fragment never change distance and only shift the energy by a constant.
 */
orc_ligand *orc_ligand_create(int n_atoms, const float *xyz, const int *types, int n_frags,
                              const int *frag_start, const int *frag_parent, const int *axis,
                              int n_bonds, const int *bonds)
{
    if (n_atoms < 1 || n_atoms > ORC_MAX_ATOMS || n_frags < 1 || n_frags > ORC_MAX_FRAGS) return NULL;
    orc_ligand *L = (orc_ligand *)calloc(1, sizeof(orc_ligand));
    L->n_atoms = n_atoms; L->n_frags = n_frags; L->n_tors = n_frags - 1;
    for (int i = 0; i < n_atoms; i++) {
        for (int a = 0; a < 3; a++) L->ref[i][a] = (double)xyz[3 * i + a];
        L->type[i] = types[i];
        if (types[i] < 0 || types[i] >= ORC_NXS) { free(L); return NULL; }
    }
    if (frag_start[0] != 0 || frag_start[n_frags] != n_atoms) { free(L); return NULL; }
    for (int k = 0; k <= n_frags; k++) L->frag_start[k] = frag_start[k];
    for (int k = 0; k < n_frags; k++) {
        if (frag_start[k + 1] <= frag_start[k]) { free(L); return NULL; }
        for (int i = frag_start[k]; i < frag_start[k + 1]; i++) L->frag_of[i] = k;
        L->parent[k] = frag_parent[k];
        if (k == 0 ? frag_parent[0] != -1 : (frag_parent[k] < 0 || frag_parent[k] >= k)) { free(L); return NULL; }
        L->axis_a[k] = k ? axis[2 * k] : -1;
        L->axis_b[k] = k ? axis[2 * k + 1] : -1;
    }
    for (int k = 1; k < n_frags; k++) {
        int a = L->axis_a[k], b = L->axis_b[k];
        if (a < 0 || a >= n_atoms || b < 0 || b >= n_atoms || L->frag_of[a] != L->parent[k] || L->frag_of[b] != k) {
            free(L); return NULL;
        }
    }
    /* root centre and gyration radius */
    int n0 = frag_start[1];
    for (int a = 0; a < 3; a++) {
        double s = 0;
        for (int i = 0; i < n0; i++) s += L->ref[i][a];
        L->root_centre[a] = s / n0;
    }
    double s2 = 0;
    for (int i = 0; i < n_atoms; i++)
        for (int a = 0; a < 3; a++) s2 += (L->ref[i][a] - L->root_centre[a]) * (L->ref[i][a] - L->root_centre[a]);
    L->rg = sqrt(s2 / n_atoms);
    /* subtree membership */
    for (int k = 0; k < n_frags; k++)
        for (int m = 0; m < n_frags; m++) {
            int x = m;
            while (x >= 0 && x != k) x = L->parent[x];
            L->in_subtree[k][m] = (x == k);
        }
    /* bond-graph distances (BFS from each atom) for the 1-2/1-3/1-4 exclusions */
    static const int INF = 1 << 20;
    int adj[ORC_MAX_ATOMS][ORC_MAX_ATOMS];
    int deg[ORC_MAX_ATOMS];
    memset(deg, 0, sizeof deg);
    for (int b = 0; b < n_bonds; b++) {
        int i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || i >= n_atoms || j < 0 || j >= n_atoms || i == j) { free(L); return NULL; }
        adj[i][deg[i]++] = j;
        adj[j][deg[j]++] = i;
    }
    for (int k = 1; k < n_frags; k++) {   /* the torsion axis must be a bond */
        int a = L->axis_a[k], b = L->axis_b[k], found = 0;
        for (int q = 0; q < deg[a]; q++) if (adj[a][q] == b) found = 1;
        if (!found) { free(L); return NULL; }
    }
    L->n_pairs = 0;
    for (int i = 0; i < n_atoms; i++) {
        int dist[ORC_MAX_ATOMS], queue[ORC_MAX_ATOMS], qh = 0, qt = 0;
        for (int j = 0; j < n_atoms; j++) dist[j] = INF;
        dist[i] = 0; queue[qt++] = i;
        while (qh < qt) {
            int u = queue[qh++];
            for (int q = 0; q < deg[u]; q++) {
                int v = adj[u][q];
                if (dist[v] == INF) { dist[v] = dist[u] + 1; queue[qt++] = v; }
            }
        }
        for (int j = i + 1; j < n_atoms; j++)
            if (L->frag_of[i] != L->frag_of[j] && dist[j] > 3) {
                L->pair_i[L->n_pairs] = i;
                L->pair_j[L->n_pairs] = j;
                L->n_pairs++;
            }
    }
    return L;
}

void orc_ligand_free(orc_ligand *L) { free(L); }
int orc_ligand_n_pairs(const orc_ligand *L) { return L->n_pairs; }
void orc_ligand_pairs(const orc_ligand *L, int *out)
{
    for (int p = 0; p < L->n_pairs; p++) { out[2 * p] = L->pair_i[p]; out[2 * p + 1] = L->pair_j[p]; }
}
double orc_ligand_rg(const orc_ligand *L) { return L->rg; }
void orc_ligand_root_centre(const orc_ligand *L, double *c) { for (int a = 0; a < 3; a++) c[a] = L->root_centre[a]; }

/* 3x3 helpers (row-major) */
static void mat_vec(const double *R, const double *v, double *o)
{
    for (int r = 0; r < 3; r++) o[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
}
static void mat_mul(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}
static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_to_mat(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
/* rotation by angle th about unit axis u (right-handed, Rodrigues) */
static void axis_angle(const double *u, double th, double *R)
{
    double c = cos(th), s = sin(th), t = 1 - c;
    R[0] = c + t * u[0] * u[0];        R[1] = t * u[0] * u[1] - s * u[2]; R[2] = t * u[0] * u[2] + s * u[1];
    R[3] = t * u[1] * u[0] + s * u[2]; R[4] = c + t * u[1] * u[1];        R[5] = t * u[1] * u[2] - s * u[0];
    R[6] = t * u[2] * u[0] - s * u[1]; R[7] = t * u[2] * u[1] + s * u[0]; R[8] = c + t * u[2] * u[2];
}

/*
 * Forward kinematics.  Pose = (p[3], q[4] = w,x,y,z, theta[n_tors]); theta_k turns
 * fragment k+1.
 *   root:   x_i = p + R(q) (ref_i - c0), c0 = centroid of the root fragment's
 *           reference atoms, so theta = 0, q = identity, p = c0 is the input
 *           conformation;
 *   child k: turns by theta about the bond a_k -> b_k of its parent's frame:
 *           R_k = R_parent * Rot(ref_u_k, theta), ref_u_k = unit(ref_b - ref_a),
 *           x_i = o_k + R_k (ref_i - ref_b_k), o_k = world position of b_k.
 * Outputs coordinates, per-fragment origins o_k (root: p) and world axes u_k.
 */
static void fk(const orc_ligand *L, const double *pose, double (*x)[3], double (*o)[3], double (*u)[3])
{
    double R[ORC_MAX_FRAGS][9];
    double q[4] = {pose[3], pose[4], pose[5], pose[6]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int c = 0; c < 4; c++) q[c] /= qn;
    quat_to_mat(q, R[0]);
    for (int a = 0; a < 3; a++) { o[0][a] = pose[a]; u[0][a] = 0; }
    for (int k = 1; k < L->n_frags; k++) {
        int par = L->parent[k], a = L->axis_a[k], b = L->axis_b[k];
        double ru[3], d[3], Q[9];
        for (int c = 0; c < 3; c++) ru[c] = L->ref[b][c] - L->ref[a][c];
        double nu = sqrt(ru[0] * ru[0] + ru[1] * ru[1] + ru[2] * ru[2]);
        for (int c = 0; c < 3; c++) ru[c] /= nu;
        axis_angle(ru, pose[7 + (k - 1)], Q);
        mat_mul(R[par], Q, R[k]);
        mat_vec(R[par], ru, u[k]);
        /* origin of k: b_k placed by the parent's frame */
        double refo_par[3];
        if (par == 0) for (int c = 0; c < 3; c++) refo_par[c] = L->root_centre[c];
        else for (int c = 0; c < 3; c++) refo_par[c] = L->ref[L->axis_b[par]][c];
        for (int c = 0; c < 3; c++) d[c] = L->ref[b][c] - refo_par[c];
        double w[3];
        mat_vec(R[par], d, w);
        for (int c = 0; c < 3; c++) o[k][c] = o[par][c] + w[c];
    }
    for (int i = 0; i < L->n_atoms; i++) {
        int k = L->frag_of[i];
        double refo[3], d[3], w[3];
        if (k == 0) for (int c = 0; c < 3; c++) refo[c] = L->root_centre[c];
        else for (int c = 0; c < 3; c++) refo[c] = L->ref[L->axis_b[k]][c];
        for (int c = 0; c < 3; c++) d[c] = L->ref[i][c] - refo[c];
        mat_vec(R[k], d, w);
        for (int c = 0; c < 3; c++) x[i][c] = o[k][c] + w[c];
    }
}

void orc_fk(const orc_ligand *L, const double *pose, double *xyz)
{
    double x[ORC_MAX_ATOMS][3], o[ORC_MAX_FRAGS][3], u[ORC_MAX_FRAGS][3];
    fk(L, pose, x, o, u);
    memcpy(xyz, x, sizeof(double) * 3 * L->n_atoms);
}

/* ------------------------------------------------------------------------- */
/* Pose energy and gradient.                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    const double *xyz;    /* [n][3] */
    const int *type;
    int n;
} orc_receptor;

orc_receptor *orc_receptor_create(const double *xyz, const int *type, int n)
{
    orc_receptor *r = (orc_receptor *)calloc(1, sizeof(orc_receptor));
    r->xyz = xyz; r->type = type; r->n = n;
    return r;
}
void orc_receptor_free(orc_receptor *r) { free(r); }

/*
 * Energy of a pose and its gradient in the tangent coordinates
 *   (dp[3], rotation vector w[3] applied as q <- quat(w) * q, dtheta[n_tors]).
 * e_total = E_inter + E_intra, where E_inter includes the wall (and, with site
 * points, the restraint of the root position to the adaptive search space).
 *   mode EQ4 / EQ3: inter-molecular part from the maps (eq. 2 energy; eq. 4 or
 *   eq. 3 gradient).  mode DIRECT: from the receptor atoms by direct summation
 *   (grid-free), with the same wall; used to check gradients by finite differences.
 * Per-atom forces f_i = dE/dx_i are carried to the pose coordinates:
 *   dE/dp = sum f_i;  dE/dw = sum (x_i - p) x f_i;
 *   dE/dtheta_k = u_k . sum_{i in subtree(k)} (x_i - o_k) x f_i.
 * parts (nullable) = {E_inter (incl. wall), E_intra, wall, e_total}.
 * mass (nullable) = {energy mass, gradient mass, energy tie, gradient tie}:
 *   sums of absolute contributions and near-tie contributions, used by tests to
 *   scale tolerances.
 */
double orc_eval(const orc_ligand *L, const orc_grid *g, const orc_receptor *rec, int mode, const double *pose,
                double wall_slope, double *grad, double *parts, double *xyz_out, double *mass, double tie_eps)
{
    double x[ORC_MAX_ATOMS][3], o[ORC_MAX_FRAGS][3], u[ORC_MAX_FRAGS][3], f[ORC_MAX_ATOMS][3];
    fk(L, pose, x, o, u);
    double e_inter = 0, e_intra = 0, wall = 0, me = 0, mg = 0, te = 0, tg = 0;
    for (int i = 0; i < L->n_atoms; i++) {
        double e, gr[3], w = 0;
        if (mode == ORC_MODE_DIRECT) {
            double out[4], ms[2], ti[2];
            direct_point(rec->xyz, rec->type, rec->n, L->type[i], x[i], out, ms, ti, tie_eps);
            /* the same wall as the grid modes: energy outside the box, clamped axes see only the wall */
            double gw[3] = {0, 0, 0};
            for (int a = 0; a < 3; a++) {
                double lo = g->origin[a], hi = g->origin[a] + (g->n[a] - 1) * g->h;
                if (x[i][a] < lo) { w += wall_slope * (lo - x[i][a]); gw[a] = -wall_slope; }
                else if (x[i][a] > hi) { w += wall_slope * (x[i][a] - hi); gw[a] = wall_slope; }
            }
            if (w > 0) {
                /* outside the box the direct energy is taken at the clamped point */
                double xc[3];
                for (int a = 0; a < 3; a++) {
                    double lo = g->origin[a], hi = g->origin[a] + (g->n[a] - 1) * g->h;
                    xc[a] = x[i][a] < lo ? lo : (x[i][a] > hi ? hi : x[i][a]);
                }
                direct_point(rec->xyz, rec->type, rec->n, L->type[i], xc, out, ms, ti, tie_eps);
                for (int a = 0; a < 3; a++) if (gw[a] != 0) out[1 + a] = 0;
            }
            e = out[0] + w;
            for (int a = 0; a < 3; a++) gr[a] = out[1 + a] + gw[a];
            me += ms[0] + w; mg += ms[1]; te += ti[0]; tg += ti[1];
        } else {
            int t = g->map_of_type[L->type[i]];
            double ms[2] = {0, 0}, ti[2] = {0, 0};
            interp(g, t, x[i], mode, wall_slope, &e, gr, &w, ms, ti, tie_eps);
            me += ms[0]; mg += ms[1]; te += ti[0]; tg += ti[1];
        }
        e_inter += e;
        wall += w;
        for (int a = 0; a < 3; a++) f[i][a] = gr[a];
    }
    for (int p = 0; p < L->n_pairs; p++) {
        int i = L->pair_i[p], j = L->pair_j[p];
        double d[3] = {x[i][0] - x[j][0], x[i][1] - x[j][1], x[i][2] - x[j][2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double a, b;
        pair_tie(L->type[i], L->type[j], r, tie_eps, &a, &b);
        te += a; tg += 2 * b;
        if (r >= ORC_CUTOFF) continue;
        double dd;
        e_intra += orc_pair_energy(L->type[i], L->type[j], r, &dd);
        pair_mass(L->type[i], L->type[j], r, &a, &b);
        me += a; mg += 2 * b;
        if (r > 1e-9)
            for (int c = 0; c < 3; c++) { f[i][c] += dd * d[c] / r; f[j][c] -= dd * d[c] / r; }
    }
    double gsite[3] = {0, 0, 0};
    const double e_site = orc_site_term(g, pose, wall_slope, gsite);
    e_inter += e_site;
    wall += e_site;
    me += e_site;
    if (e_site > 0) mg += wall_slope;
    double E = e_inter + e_intra;
    if (grad) {
        double F[3] = {gsite[0], gsite[1], gsite[2]}, tq[3] = {0, 0, 0};
        for (int i = 0; i < L->n_atoms; i++) {
            double rel[3] = {x[i][0] - pose[0], x[i][1] - pose[1], x[i][2] - pose[2]}, c[3];
            cross(rel, f[i], c);
            for (int a = 0; a < 3; a++) { F[a] += f[i][a]; tq[a] += c[a]; }
        }
        for (int a = 0; a < 3; a++) { grad[a] = F[a]; grad[3 + a] = tq[a]; }
        for (int k = 1; k < L->n_frags; k++) {
            double tk[3] = {0, 0, 0};
            for (int i = 0; i < L->n_atoms; i++) {
                if (!L->in_subtree[k][L->frag_of[i]]) continue;
                double rel[3] = {x[i][0] - o[k][0], x[i][1] - o[k][1], x[i][2] - o[k][2]}, c[3];
                cross(rel, f[i], c);
                for (int a = 0; a < 3; a++) tk[a] += c[a];
            }
            grad[6 + (k - 1)] = u[k][0] * tk[0] + u[k][1] * tk[1] + u[k][2] * tk[2];
        }
    }
    if (parts) { parts[0] = e_inter; parts[1] = e_intra; parts[2] = wall; parts[3] = E; }
    if (xyz_out) memcpy(xyz_out, x, sizeof(double) * 3 * L->n_atoms);
    if (mass) { mass[0] = me; mass[1] = mg; mass[2] = te; mass[3] = tg; }
    return E;
}

/* ------------------------------------------------------------------------- */
/* Pose increments.                                                           */
/* ------------------------------------------------------------------------- */

/* unit quaternion of the rotation vector v: angle |v| about v/|v| */
static void quat_of_rotvec(const double *v, double *q)
{
    double a = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (a == 0) { q[0] = 1; q[1] = q[2] = q[3] = 0; return; }
    double s = sin(0.5 * a) / a;
    q[0] = cos(0.5 * a); q[1] = s * v[0]; q[2] = s * v[1]; q[3] = s * v[2];
}
/* Hamilton product a*b */
static void quat_mul(const double *a, const double *b, double *o)
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}
/* into (-pi, pi]; non-finite values pass through, huge ones are reduced first */
static double wrap_angle(double t)
{
    if (!isfinite(t)) return t;
    if (fabs(t) > 1.0e4) t = fmod(t, 2 * ORC_PI);
    while (t > ORC_PI) t -= 2 * ORC_PI;
    while (t <= -ORC_PI) t += 2 * ORC_PI;
    return t;
}

/* pose (+) step:  p += dp;  q <- normalise(quat(w) * q);  theta <- wrap(theta + dtheta) */
void orc_pose_step(const orc_ligand *L, const double *pose, const double *step, double *out)
{
    double dq[4], q[4], nq[4];
    for (int a = 0; a < 3; a++) out[a] = pose[a] + step[a];
    quat_of_rotvec(step + 3, dq);
    for (int c = 0; c < 4; c++) q[c] = pose[3 + c];
    quat_mul(dq, q, nq);
    double n = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
    for (int c = 0; c < 4; c++) out[3 + c] = nq[c] / n;
    for (int k = 0; k < L->n_tors; k++) out[7 + k] = wrap_angle(pose[7 + k] + step[6 + k]);
}

/* ------------------------------------------------------------------------- */
/* BFGS with Armijo backtracking (Nocedal & Wright, ref. [36]).               */
/* ------------------------------------------------------------------------- */

#define ORC_OPT_BFGS 0
#define ORC_OPT_BB 1

typedef struct {
    double temperature, wall_slope, rmsd_cluster, trans_amp;
    int bfgs_iters, ls_trials;
    double ls_shrink, armijo_c1;
    int optimizer;            /* ORC_OPT_BFGS or ORC_OPT_BB */
    int bb_iters;             /* Barzilai-Borwein iterations */
    double bb_step0;          /* first BB step length (and the one used when s.y <= 0) */
    double bb_step_max;       /* largest BB step length */
    double ls_min_decrease;   /* smallest energy decrease a line-search trial must reach */
} orc_params;

void orc_params_default(orc_params *p)
{
    p->temperature = 1.2;   /* Vina's Metropolis temperature */
    p->wall_slope = 10.0;
    p->rmsd_cluster = 1.0;
    p->trans_amp = 2.0;     /* Vina's mutation amplitude (A) */
    p->bfgs_iters = 20;
    p->ls_trials = 10;
    p->ls_shrink = 0.1;
    p->armijo_c1 = 1e-4;
    p->optimizer = ORC_OPT_BFGS;
    p->bb_iters = 100;        /* the paper finds 100-150 BB iterations enough (Section 2, Figure 2) */
    p->bb_step0 = 1e-2;
    p->bb_step_max = 1.0;
    p->ls_min_decrease = 1e-4;
}

/* generic objective: returns f(x), writes g = grad f(x) (dimension D) */
typedef double (*orc_objective)(void *ctx, const double *x, double *g);
/* generic retraction: x_new = x (+) step */
typedef void (*orc_retract)(void *ctx, const double *x, const double *step, double *x_new);

#define ORC_MAXD 40
#define ORC_MAXX 48

/*
 * Inverse-BFGS update of the D x D matrix H (row stride ORC_MAXD) with the step s
 * and gradient change y, y.s > 0 (Nocedal & Wright, ref. [36]):
 *   H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T,  rho = 1 / y.s,
 * written out for a symmetric H as
 *   H + rho ((1 + rho y^T H y) s s^T - s (H y)^T - (H y) s^T).
 * The result satisfies the secant condition H y = s.
 */
void orc_bfgs_update(int D, double *H, const double *s, const double *y)
{
    double Hy[ORC_MAXD], ys = 0, yHy = 0;
    for (int r = 0; r < D; r++) ys += y[r] * s[r];
    const double rho = 1.0 / ys;
    for (int r = 0; r < D; r++) {
        double acc = 0;
        for (int c = 0; c < D; c++) acc += H[r * ORC_MAXD + c] * y[c];
        Hy[r] = acc;
        yHy += y[r] * acc;
    }
    for (int r = 0; r < D; r++)
        for (int c = 0; c < D; c++)
            H[r * ORC_MAXD + c] += rho * ((1.0 + rho * yHy) * s[r] * s[c] - s[r] * Hy[c] - Hy[r] * s[c]);
}

/*
 * Inverse-BFGS minimisation in tangent coordinates.
 *   H = I; repeat `iters` times:
 *     p = -H g;  line search: alpha = 1, shrink by `shrink` up to `trials` times
 *     until f(x (+) alpha p) - f(x) <= min(c1 alpha g.p, -min_dec) (the Armijo
 *     test, with a decrease of at least min_dec); none accepted -> stop;
 *     s = alpha p, y = g_new - g; if y.s > 0: inverse-BFGS update of H.
 * x has dimension nx (the pose, with a 4-component quaternion), the tangent
 * space dimension D.  Returns the number of objective evaluations.  margin
 * (nullable) receives the smallest relative distance of any line-search or
 * curvature test from its threshold (how close the run came to a different
 * decision).
 */
long orc_bfgs(void *ctx, orc_objective f, orc_retract retract, int nx, int D, double *x, double *fx, double *g,
              int iters, int trials, double shrink, double c1, double min_dec, double *margin)
{
    double H[ORC_MAXD][ORC_MAXD], p[ORC_MAXD], gn[ORC_MAXD], s[ORC_MAXD], y[ORC_MAXD];
    double xn[ORC_MAXX], step[ORC_MAXD];
    long evals = 0;
    double mmin = DBL_MAX;
    double E = f(ctx, x, g);
    evals++;
    for (int r = 0; r < D; r++) for (int c = 0; c < D; c++) H[r][c] = (r == c);
    for (int it = 0; it < iters; it++) {
        double gp = 0;
        for (int r = 0; r < D; r++) {
            double acc = 0;
            for (int c = 0; c < D; c++) acc += H[r][c] * g[c];
            p[r] = -acc;
            gp += p[r] * g[r];
        }
        double alpha = 1.0, En = 0;
        int ok = 0;
        for (int t = 0; t < trials; t++) {
            for (int r = 0; r < D; r++) step[r] = alpha * p[r];
            retract(ctx, x, step, xn);
            En = f(ctx, xn, gn);
            evals++;
            double thr = fmin(c1 * alpha * gp, -min_dec);
            double rel = fabs((En - E) - thr) / (fabs(E) + fabs(E + thr) + 1e-12);
            if (rel < mmin) mmin = rel;
            if (En - E <= thr) { ok = 1; break; }
            alpha *= shrink;
        }
        if (!ok) break;
        double ys = 0, ss = 0, yy = 0;
        for (int r = 0; r < D; r++) {
            s[r] = alpha * p[r];
            y[r] = gn[r] - g[r];
            ys += y[r] * s[r];
            ss += s[r] * s[r];
            yy += y[r] * y[r];
        }
        memcpy(x, xn, sizeof(double) * nx);
        memcpy(g, gn, sizeof(double) * D);
        E = En;
        double crel = fabs(ys) / (sqrt(ss * yy) + 1e-300);
        if (crel < mmin) mmin = crel;
        if (ys > 0) orc_bfgs_update(D, &H[0][0], s, y);
    }
    *fx = E;
    if (margin) *margin = mmin;
    return evals;
}

/* ------------------------------------------------------------------------- */
/* Barzilai-Borwein gradient method (Section 2, "Binding pose search", second */
/* modification; ref. [37]): no line search, the step length from the last   */
/* step and gradient change.                                                  */
/* ------------------------------------------------------------------------- */

/*
 *   g = grad f(x); a = step0; best = (f(x), x)
 *   repeat `iters` times:
 *     s = -a g;  x <- x (+) s;  g_new = grad f(x);  y = g_new - g;  g <- g_new
 *     a = s.s / s.y if s.y > 0 (capped at step_max), else step0
 *     best <- (f(x), x) if f(x) < best energy
 *   return best (the method does not decrease f monotonically).
 * Returns the number of objective evaluations (iters + 1).  g receives the
 * gradient at the returned point.
 */
long orc_bb(void *ctx, orc_objective f, orc_retract retract, int nx, int D, double *x, double *fx, double *g,
            int iters, double step0, double step_max, double *margin)
{
    double s[ORC_MAXD], gn[ORC_MAXD], xn[ORC_MAXX], xb[ORC_MAXX], gb[ORC_MAXD];
    long evals = 0;
    double mmin = DBL_MAX;
    double E = f(ctx, x, g);
    evals++;
    double Eb = E;
    memcpy(xb, x, sizeof(double) * nx);
    memcpy(gb, g, sizeof(double) * D);
    double a = step0;
    for (int it = 0; it < iters; it++) {
        for (int r = 0; r < D; r++) s[r] = -a * g[r];
        retract(ctx, x, s, xn);
        double En = f(ctx, xn, gn);
        evals++;
        double sy = 0, ss = 0, yy = 0;
        for (int r = 0; r < D; r++) {
            sy += s[r] * (gn[r] - g[r]);
            ss += s[r] * s[r];
            yy += (gn[r] - g[r]) * (gn[r] - g[r]);
        }
        a = sy > 0 ? fmin(ss / sy, step_max) : step0;
        /* closeness of each decision to its threshold: the sign of s.y, the cap,
           and the best-iterate comparison */
        double m = fabs(sy) / (sqrt(ss * yy) + 1e-300);
        if (sy > 0) m = fmin(m, fabs(ss / sy - step_max) / step_max);
        m = fmin(m, fabs(En - Eb) / (fabs(En) + fabs(Eb) + 1e-12));
        if (m < mmin) mmin = m;
        memcpy(x, xn, sizeof(double) * nx);
        memcpy(g, gn, sizeof(double) * D);
        if (En < Eb) {
            Eb = En;
            memcpy(xb, xn, sizeof(double) * nx);
            memcpy(gb, gn, sizeof(double) * D);
        }
    }
    memcpy(x, xb, sizeof(double) * nx);
    memcpy(g, gb, sizeof(double) * D);
    *fx = Eb;
    if (margin) *margin = mmin;
    return evals;
}

typedef struct {
    const orc_ligand *L;
    const orc_grid *g;
    const orc_receptor *rec;
    int mode;
    double wall_slope;
} pose_ctx;

static double pose_objective(void *vctx, const double *x, double *g)
{
    pose_ctx *c = (pose_ctx *)vctx;
    return orc_eval(c->L, c->g, c->rec, c->mode, x, c->wall_slope, g, NULL, NULL, NULL, 0);
}
static void pose_retract(void *vctx, const double *x, const double *step, double *xn)
{
    pose_ctx *c = (pose_ctx *)vctx;
    orc_pose_step(c->L, x, step, xn);
}

/*
 * Local optimisation of one pose (eq. 4 gradients, the search mode).
 * pose is updated in place; returns the evaluation count.
 */
long orc_local_opt(const orc_ligand *L, const orc_grid *g, const orc_params *prm, double *pose, double *E,
                   double *grad, double *margin)
{
    pose_ctx c = {L, g, NULL, ORC_MODE_EQ4, prm->wall_slope};
    double gl[ORC_MAXD];
    long n;
    if (prm->optimizer == ORC_OPT_BB) {
        n = orc_bb(&c, pose_objective, pose_retract, 7 + L->n_tors, 6 + L->n_tors, pose, E, gl, prm->bb_iters,
                   prm->bb_step0, prm->bb_step_max, margin);
    } else {
        n = orc_bfgs(&c, pose_objective, pose_retract, 7 + L->n_tors, 6 + L->n_tors, pose, E, gl,
                     prm->bfgs_iters, prm->ls_trials, prm->ls_shrink, prm->armijo_c1, prm->ls_min_decrease, margin);
    }
    if (grad) memcpy(grad, gl, sizeof(double) * (6 + L->n_tors));
    return n;
}

/* generic BFGS over a ctypes callback, for textbook-function pins */
typedef struct { orc_objective f; int D; } plain_ctx;
static double plain_objective(void *vctx, const double *x, double *g)
{
    plain_ctx *c = (plain_ctx *)vctx;
    return c->f(NULL, x, g);
}
static void plain_retract(void *vctx, const double *x, const double *step, double *xn)
{
    plain_ctx *c = (plain_ctx *)vctx;
    for (int r = 0; r < c->D; r++) xn[r] = x[r] + step[r];
}
long orc_bfgs_plain(orc_objective f, int D, double *x, double *fx, double *g, int iters, int trials, double shrink,
                    double c1, double min_dec)
{
    plain_ctx c = {f, D};
    return orc_bfgs(&c, plain_objective, plain_retract, D, D, x, fx, g, iters, trials, shrink, c1, min_dec, NULL);
}

/* generic Barzilai-Borwein over a ctypes callback, for textbook-function pins */
long orc_bb_plain(orc_objective f, int D, double *x, double *fx, double *g, int iters, double step0, double step_max)
{
    plain_ctx c = {f, D};
    return orc_bb(&c, plain_objective, plain_retract, D, D, x, fx, g, iters, step0, step_max, NULL);
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its        */
/* definition: 10 rounds of two 32x32->64 multiplies with a Weyl key schedule. */
/* ------------------------------------------------------------------------- */

void orc_philox(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c[0];
        uint64_t p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    for (int i = 0; i < 4; i++) out[i] = c[i];
}

/* uniform in [0, 1) from the top 24 bits: exact in single and double precision */
static double unif(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* random-number streams of one chain: counter = (chain, step, stream, block), key = seed */
enum { ORC_TAG_INIT = 0, ORC_TAG_MUTATE = 1, ORC_TAG_METROPOLIS = 2, ORC_TAG_SITE = 3 };
#define ORC_SITE_ATTEMPTS 64

static void draw(uint64_t seed, uint32_t chain, uint32_t step, uint32_t tag, uint32_t block, uint32_t *out)
{
    uint32_t ctr[4] = {chain, step, tag, block};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* point in the unit ball: direction from (z = 2u1 - 1, phi = 2 pi u2), radius u3^(1/3) */
void orc_ball(double u1, double u2, double u3, double *v)
{
    double z = 2 * u1 - 1, phi = 2 * ORC_PI * u2, r = cbrt(u3);
    double s = sqrt(fmax(0.0, 1 - z * z));
    v[0] = r * s * cos(phi); v[1] = r * s * sin(phi); v[2] = r * z;
}

/* uniform random rotation (Shoemake's method) as (w, x, y, z) */
void orc_shoemake(double u1, double u2, double u3, double *q)
{
    double s1 = sqrt(1 - u1), s2 = sqrt(u1), a = 2 * ORC_PI * u2, b = 2 * ORC_PI * u3;
    q[1] = s1 * sin(a); q[2] = s1 * cos(a); q[3] = s2 * sin(b); q[0] = s2 * cos(b);
}

/* Initial pose of a chain: position uniform in the box, uniform orientation, torsions uniform in [-pi, pi). */
void orc_initial_pose(const orc_ligand *L, const orc_grid *g, uint64_t seed, uint32_t chain, double *pose)
{
    int nw = 6 + L->n_tors;
    double u[6 + ORC_MAX_FRAGS];
    for (int w = 0; w < nw; w += 4) {
        uint32_t r[4];
        draw(seed, chain, 0, ORC_TAG_INIT, (uint32_t)(w / 4), r);
        for (int c = 0; c < 4 && w + c < nw; c++) u[w + c] = unif(r[c]);
    }
    for (int a = 0; a < 3; a++) pose[a] = g->origin[a] + u[a] * (g->n[a] - 1) * g->h;
    if (g->n_site > 0) {
        /* adaptive search space: the first of up to ORC_SITE_ATTEMPTS uniform points
           of the box (one Philox block each) that lies in a site ball; none: the
           first site point */
        int ok = 0;
        for (uint32_t k = 0; k < ORC_SITE_ATTEMPTS && !ok; k++) {
            uint32_t r[4];
            draw(seed, chain, 0, ORC_TAG_SITE, k, r);
            double c[3];
            for (int a = 0; a < 3; a++) c[a] = g->origin[a] + unif(r[a]) * (g->n[a] - 1) * g->h;
            for (int i = 0; i < g->n_site && !ok; i++) {
                double d2 = 0;
                for (int a = 0; a < 3; a++) d2 += (c[a] - g->site[3 * i + a]) * (c[a] - g->site[3 * i + a]);
                if (d2 <= g->site_r * g->site_r) ok = 1;
            }
            if (ok)
                for (int a = 0; a < 3; a++) pose[a] = c[a];
        }
        if (!ok)
            for (int a = 0; a < 3; a++) pose[a] = g->site[a];
    }
    orc_shoemake(u[3], u[4], u[5], pose + 3);
    for (int k = 0; k < L->n_tors; k++) pose[7 + k] = -ORC_PI + 2 * ORC_PI * u[6 + k];
}

/*
 * Mutation at MC step `step` (Vina's move set, ref. [6]): one of 2 + n_tors moves
 * chosen uniformly:
 *   0: translate by trans_amp * (point in the unit ball);
 *   1: rotate by the rotation vector (trans_amp / Rg) * (point in the unit ball);
 *   2 + k: set torsion k to a uniform angle in [-pi, pi).
 * The choice is the integer floor(x0 * (2 + n_tors) / 2^32), so both sides take
 * it in integer arithmetic.  Returns the move index.
 */
int orc_mutate(const orc_ligand *L, const orc_params *prm, uint64_t seed, uint32_t chain, uint32_t step, double *pose)
{
    uint32_t r[4];
    draw(seed, chain, step, ORC_TAG_MUTATE, 0, r);
    int which = (int)(((uint64_t)r[0] * (uint64_t)(2 + L->n_tors)) >> 32);
    double u1 = unif(r[1]), u2 = unif(r[2]), u3 = unif(r[3]);
    if (which == 0) {
        double v[3];
        orc_ball(u1, u2, u3, v);
        for (int a = 0; a < 3; a++) pose[a] += prm->trans_amp * v[a];
    } else if (which == 1) {
        double v[3], dq[4], q[4], nq[4];
        orc_ball(u1, u2, u3, v);
        double amp = L->rg > 0 ? prm->trans_amp / L->rg : 0.0;
        for (int a = 0; a < 3; a++) v[a] *= amp;
        quat_of_rotvec(v, dq);
        for (int c = 0; c < 4; c++) q[c] = pose[3 + c];
        quat_mul(dq, q, nq);
        double n = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
        for (int c = 0; c < 4; c++) pose[3 + c] = nq[c] / n;
    } else {
        pose[7 + (which - 2)] = -ORC_PI + 2 * ORC_PI * u1;
    }
    return which;
}

/* Metropolis acceptance (ref. [6]): accept if dE < 0 or u < exp(-dE / T). */
int orc_metropolis(double e_new, double e_old, double T, double u)
{
    double dE = e_new - e_old;
    if (dE < 0) return 1;
    return u < exp(-dE / T);
}

double orc_metropolis_uniform(uint64_t seed, uint32_t chain, uint32_t step)
{
    uint32_t r[4];
    draw(seed, chain, step, ORC_TAG_METROPOLIS, 0, r);
    return unif(r[0]);
}

/*
 * One Monte Carlo chain (Section 2, parallelisation paragraph: many copies, short
 * runs, each independent):
 *   x = initial pose; for step s = 0 .. n_steps-1:
 *     cand = local_opt(mutate(x));  accept cand if s == 0 or Metropolis(T);
 *     keep the lowest accepted energy as the chain best.
 * best_pose [7 + n_tors]; best_e = {e_total, e_inter, e_intra, wall}.
 * counters = {pose evaluations, local optimisations, acceptances}.
 */
void orc_chain(const orc_ligand *L, const orc_grid *g, const orc_params *prm, uint64_t seed, uint32_t chain,
               int n_steps, double *best_pose, double *best_e, long *counters)
{
    const int nx = 7 + L->n_tors;
    double x[ORC_MAXX], cand[ORC_MAXX], gr[ORC_MAXD];
    double Ex = 0;
    long evals = 0, lopt = 0, acc = 0;
    orc_initial_pose(L, g, seed, chain, x);
    best_e[0] = INFINITY;
    memcpy(best_pose, x, sizeof(double) * nx);
    for (int s = 0; s < n_steps; s++) {
        memcpy(cand, x, sizeof(double) * nx);
        orc_mutate(L, prm, seed, chain, (uint32_t)s, cand);
        double Ec;
        evals += orc_local_opt(L, g, prm, cand, &Ec, gr, NULL);
        lopt++;
        int take = (s == 0) ? 1 : orc_metropolis(Ec, Ex, prm->temperature, orc_metropolis_uniform(seed, chain, (uint32_t)s));
        if (take) {
            memcpy(x, cand, sizeof(double) * nx);
            Ex = Ec;
            acc++;
            if (Ex < best_e[0]) {
                double parts[4];
                orc_eval(L, g, NULL, ORC_MODE_EQ4, x, prm->wall_slope, NULL, parts, NULL, NULL, 0);
                memcpy(best_pose, x, sizeof(double) * nx);
                best_e[0] = Ex; best_e[1] = parts[0]; best_e[2] = parts[1]; best_e[3] = parts[2];
            }
        }
    }
    counters[0] = evals; counters[1] = lopt; counters[2] = acc;
}

/* All chains of one dock, OpenMP over chains (they are independent). */
void orc_dock(const orc_ligand *L, const orc_grid *g, const orc_params *prm, int n_chains, int n_steps,
              uint64_t seed, double *best_pose, double *best_e, long *counters, int n_threads)
{
    const int nx = 7 + L->n_tors;
#ifdef _OPENMP
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int c = 0; c < n_chains; c++)
        orc_chain(L, g, prm, seed, (uint32_t)c, n_steps, best_pose + (long)c * nx, best_e + 4L * c, counters + 3L * c);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Post-processing: ranking and RMSD clustering (Section 2 parallelisation     */
/* paragraph: poses are post-processed on the CPU; heavy-atom RMSD, Section 2  */
/* "Baseline Setup").                                                         */
/* ------------------------------------------------------------------------- */

/* heavy-atom RMSD between two conformations with the same atom order (no symmetry correction) */
double orc_rmsd(const double *a, const double *b, int n)
{
    double s = 0;
    for (int i = 0; i < 3 * n; i++) s += (a[i] - b[i]) * (a[i] - b[i]);
    return sqrt(s / n);
}

/*
 * Ranking reading: candidates ordered by e_total (ties by chain index); a pose
 * is kept if its RMSD to every pose kept before it exceeds `cut`; stop at k.
 * Non-finite energies are skipped.  xyz: [C][n_atoms][3].  Returns the count.
 */
int orc_topk(const double *energy, const double *xyz, int n_atoms, int C, int k, double cut, int *out_idx)
{
    int *order = (int *)malloc(sizeof(int) * (C > 0 ? C : 1));
    int m = 0;
    for (int c = 0; c < C; c++) if (isfinite(energy[c])) order[m++] = c;
    /* insertion sort by (energy, index): plain and stable */
    for (int a = 1; a < m; a++) {
        int v = order[a], b = a - 1;
        while (b >= 0 && (energy[order[b]] > energy[v] || (energy[order[b]] == energy[v] && order[b] > v))) {
            order[b + 1] = order[b];
            b--;
        }
        order[b + 1] = v;
    }
    int n = 0;
    for (int a = 0; a < m && n < k; a++) {
        int c = order[a], keep = 1;
        for (int q = 0; q < n; q++)
            if (orc_rmsd(xyz + (long)c * 3 * n_atoms, xyz + (long)out_idx[q] * 3 * n_atoms, n_atoms) <= cut) {
                keep = 0;
                break;
            }
        if (keep) out_idx[n++] = c;
    }
    free(order);
    return n;
}

/* Vina's reported score: inter-molecular energy over (1 + w_rot * N_rot). */
double orc_score(double e_inter, int n_tors) { return e_inter / (1.0 + W_ROT * n_tors); }
