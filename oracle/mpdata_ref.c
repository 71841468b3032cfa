/*
 * mpdata_ref.c -- plain, slow CPU FP64 oracle of one MPDATA step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the GPU path includes, links or calls
 * this file; it shares no code, header, table or helper with that path.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark load
 * it.  It is built with -O2 -ffp-contract=off (no FMA contraction, no
 * fast-math), and every expression is evaluated exactly as parenthesised.
 * It is neither tiled nor fused: every stage is a full-array loop, in the
 * order of the scheme.  The only parallelism is an OpenMP loop over levels.
 *
 * Stages and where they come from:
 *   C1 donor-cell flux        paper, Section 5, Listings 4-5 (edge flux with
 *                             max(0,v) / min(0,v) weights) and Listings 6-7
 *                             (the same along the vertical, boundary factor 0)
 *   C2 divergence and update  paper, Section 5, Listing 8 (flux, vertical
 *                             flux, flux divergence over the cell's metric
 *                             volume, solution update)
 *   C3 antidiffusive velocity MPDATA literature (the paper refers the rest
 *   C4 limiter bounds, beta   of the scheme to another deliverable): the
 *   C5 limited velocities     antidiffusive pseudo-velocity of Smolarkiewicz
 *   C6 corrective pass        (1984) in the metric form of Smolarkiewicz &
 *                             Margolin (1998), limited as in Smolarkiewicz &
 *                             Grabowski (1990)
 *   C7 mass                   sum(G psi), Neumaier compensated summation
 */
#include "mpdata_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define DEFAULT_EPS 1e-15

/* ------------------------------------------------------------------ */
/* Index helpers                                                      */
/* ------------------------------------------------------------------ */

static int64_t lin(const ref_problem* p, int i, int j, int k)
{
    return ((int64_t)k * p->ny + j) * p->nx + i;
}

static int extent(const ref_problem* p, int axis)
{
    return axis == 0 ? p->nx : (axis == 1 ? p->ny : p->nz);
}

/* Cell index along an axis with the halo rule: periodic wraps, closed clamps
 * (a zero-gradient halo). */
static int cell_index(const ref_problem* p, int axis, int i)
{
    int n = extent(p, axis);
    if (p->bc[axis] == REF_PERIODIC) return ((i % n) + n) % n;
    if (i < 0) return 0;
    if (i > n - 1) return n - 1;
    return i;
}

/* Cell value a(c) with the halo rule applied on every axis. */
static double cellv(const ref_problem* p, const double* a, const int c[3])
{
    int i = cell_index(p, 0, c[0]);
    int j = cell_index(p, 1, c[1]);
    int k = cell_index(p, 2, c[2]);
    return a[lin(p, i, j, k)];
}

/* Face value on axis `axis`: face (c[axis] + 1/2), the other two coordinates
 * being cell coordinates (halo rule applied).  On a closed axis the faces
 * -1/2 and n-1/2 (and anything beyond) carry 0; on a periodic axis the face
 * index wraps. */
static double facev(const ref_problem* p, const double* a, int axis, const int c[3])
{
    int d[3];
    for (int b = 0; b < 3; ++b)
        d[b] = (b == axis) ? c[b] : cell_index(p, b, c[b]);
    int n = extent(p, axis);
    if (p->bc[axis] == REF_CLOSED) {
        if (d[axis] <= -1 || d[axis] >= n - 1) return 0.0;
    } else {
        d[axis] = ((d[axis] % n) + n) % n;
    }
    return a[lin(p, d[0], d[1], d[2])];
}

/* Is face (c[axis] + 1/2) with 0 <= c[axis] < n a closed-boundary face? */
static int is_wall_face(const ref_problem* p, int axis, int ia)
{
    return p->bc[axis] == REF_CLOSED && ia == extent(p, axis) - 1;
}

static double pos(double c) { return c > 0.0 ? c : 0.0; }   /* [c]+ */
static double neg(double c) { return c < 0.0 ? c : 0.0; }   /* [c]- */
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

static int valid(const ref_problem* p)
{
    if (!p) return 0;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
    for (int a = 0; a < 3; ++a)
        if (p->bc[a] != REF_PERIODIC && p->bc[a] != REF_CLOSED) return 0;
    if (p->iters < 1) return 0;
    if (p->limiter != 0 && p->limiter != 1) return 0;
    if (p->eps < 0.0) return 0;
    return 1;
}

static double eps_of(const ref_problem* p)
{
    return p->eps > 0.0 ? p->eps : DEFAULT_EPS;
}

static int64_t ncells(const ref_problem* p)
{
    return (int64_t)p->nx * p->ny * p->nz;
}

/* ------------------------------------------------------------------ */
/* C1-C2: donor-cell pass                                             */
/* ------------------------------------------------------------------ */

/* C1: upwind flux through a face whose normal points from the cell with
 * value pl to the cell with value pr (paper, Listing 5 and Listing 7). */
static double donor(double pl, double pr, double c)
{
    return (pos(c) * pl) + (neg(c) * pr);
}

int ref_donor(const ref_problem* p, const double* phi, const double* u,
              const double* v, const double* w, const double* g, double* out)
{
    if (!valid(p) || !phi || !u || !v || !w || !g || !out) return -1;
    const double* vel[3] = {u, v, w};
    int64_t n = ncells(p);
    double* flx[3];
    for (int a = 0; a < 3; ++a) {
        flx[a] = (double*)malloc(sizeof(double) * (size_t)n);
        if (!flx[a]) {
            for (int b = 0; b < a; ++b) free(flx[b]);
            return -1;
        }
    }

    /* Fluxes through the three "own" faces (+1/2 side) of every cell. */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int c[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    int r[3] = {i, j, k};
                    r[a] += 1;
                    double vf = facev(p, vel[a], a, c);
                    flx[a][lin(p, i, j, k)] = donor(cellv(p, phi, c), cellv(p, phi, r), vf);
                }
            }

    /* Flux divergence over the metric volume and the update. */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int c[3] = {i, j, k};
                double dif[3];
                for (int a = 0; a < 3; ++a) {
                    int l[3] = {i, j, k};
                    l[a] -= 1;
                    dif[a] = facev(p, flx[a], a, c) - facev(p, flx[a], a, l);
                }
                int64_t q = lin(p, i, j, k);
                double div = ((dif[0] + dif[1]) + dif[2]);
                out[q] = phi[q] - div / g[q];
            }

    for (int a = 0; a < 3; ++a) free(flx[a]);
    return 0;
}

/* ------------------------------------------------------------------ */
/* C3: antidiffusive pseudo-velocities                                */
/* ------------------------------------------------------------------ */

/* Velocity on the face of axis t of the cell x (its +1/2 side). */
static double vel_face(const ref_problem* p, const double* const vel[3], int t, const int x[3])
{
    return facev(p, vel[t], t, x);
}

int ref_antidiff(const ref_problem* p, const double* phi, const double* u,
                 const double* v, const double* w, const double* g,
                 double* ut, double* vt, double* wt)
{
    if (!valid(p) || !phi || !u || !v || !w || !g || !ut || !vt || !wt) return -1;
    const double eps = eps_of(p);
    const double* vel[3] = {u, v, w};
    double* outv[3] = {ut, vt, wt};

#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i)
                for (int a = 0; a < 3; ++a) {
                    int L[3] = {i, j, k};
                    int64_t q = lin(p, i, j, k);
                    if (is_wall_face(p, a, L[a])) {
                        outv[a][q] = 0.0;
                        continue;
                    }
                    int R[3] = {i, j, k};
                    R[a] += 1;
                    /* transverse axes in increasing order */
                    int tr[2], nt = 0;
                    for (int b = 0; b < 3; ++b)
                        if (b != a) tr[nt++] = b;

                    double pL = cellv(p, phi, L), pR = cellv(p, phi, R);
                    double A = (pR - pL) / ((pR + pL) + eps);

                    double B[2], Vbar[2];
                    for (int s = 0; s < 2; ++s) {
                        int t = tr[s];
                        int Lp[3] = {L[0], L[1], L[2]}, Rp[3] = {R[0], R[1], R[2]};
                        int Lm[3] = {L[0], L[1], L[2]}, Rm[3] = {R[0], R[1], R[2]};
                        Lp[t] += 1; Rp[t] += 1; Lm[t] -= 1; Rm[t] -= 1;
                        double Sp = cellv(p, phi, Rp) + cellv(p, phi, Lp);
                        double Sm = cellv(p, phi, Rm) + cellv(p, phi, Lm);
                        B[s] = 0.5 * ((Sp - Sm) / ((Sp + Sm) + eps));
                        Vbar[s] = 0.25 * ((vel_face(p, vel, t, L) + vel_face(p, vel, t, R))
                                          + (vel_face(p, vel, t, Lm) + vel_face(p, vel, t, Rm)));
                    }
                    double Gf = 0.5 * (cellv(p, g, L) + cellv(p, g, R));
                    double U = facev(p, vel[a], a, L);
                    outv[a][q] = ((fabs(U) - (U * U) / Gf) * A)
                                 - ((U / Gf) * ((Vbar[0] * B[0]) + (Vbar[1] * B[1])));
                }
    return 0;
}

/* ------------------------------------------------------------------ */
/* C4: limiter bounds and coefficients                                */
/* ------------------------------------------------------------------ */

int ref_bounds(const ref_problem* p, const double* psin, const double* phi,
               double* mx, double* mn)
{
    if (!valid(p) || !psin || !phi || !mx || !mn) return -1;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int c[3] = {i, j, k};
                double hi = psin[lin(p, i, j, k)], lo = hi;
                /* the 7-point cross of both fields; order does not change the value */
                for (int f = 0; f < 2; ++f) {
                    const double* a = f == 0 ? psin : phi;
                    double s = cellv(p, a, c);
                    hi = dmax(hi, s);
                    lo = dmin(lo, s);
                    for (int ax = 0; ax < 3; ++ax)
                        for (int sg = -1; sg <= 1; sg += 2) {
                            int d[3] = {i, j, k};
                            d[ax] += sg;
                            double s2 = cellv(p, a, d);
                            hi = dmax(hi, s2);
                            lo = dmin(lo, s2);
                        }
                }
                mx[lin(p, i, j, k)] = hi;
                mn[lin(p, i, j, k)] = lo;
            }
    return 0;
}

int ref_beta(const ref_problem* p, const double* phi, const double* ut,
             const double* vt, const double* wt, const double* mx,
             const double* mn, const double* g, double* bup, double* bdn)
{
    if (!valid(p) || !phi || !ut || !vt || !wt || !mx || !mn || !g || !bup || !bdn) return -1;
    const double eps = eps_of(p);
    const double* vel[3] = {ut, vt, wt};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int c[3] = {i, j, k};
                double fin[3], fout[3];
                for (int a = 0; a < 3; ++a) {
                    int l[3] = {i, j, k}, r[3] = {i, j, k};
                    l[a] -= 1;
                    r[a] += 1;
                    double vr = facev(p, vel[a], a, c);  /* face +1/2 */
                    double vl = facev(p, vel[a], a, l);  /* face -1/2 */
                    /* fp(face) = [v]+ * phi(left), fm(face) = [v]- * phi(right) */
                    double fp_l = pos(vl) * cellv(p, phi, l);
                    double fm_l = neg(vl) * cellv(p, phi, c);
                    double fp_r = pos(vr) * cellv(p, phi, c);
                    double fm_r = neg(vr) * cellv(p, phi, r);
                    fin[a] = fp_l - fm_r;
                    fout[a] = fp_r - fm_l;
                }
                int64_t q = lin(p, i, j, k);
                double in = ((fin[0] + fin[1]) + fin[2]);
                double out = ((fout[0] + fout[1]) + fout[2]);
                bup[q] = ((mx[q] - phi[q]) * g[q]) / (in + eps);
                bdn[q] = ((phi[q] - mn[q]) * g[q]) / (out + eps);
            }
    return 0;
}

/* ------------------------------------------------------------------ */
/* C5: limited velocities                                             */
/* ------------------------------------------------------------------ */

int ref_limit(const ref_problem* p, const double* ut, const double* vt,
              const double* wt, const double* bup, const double* bdn,
              double* ul, double* vl, double* wl)
{
    if (!valid(p) || !ut || !vt || !wt || !bup || !bdn || !ul || !vl || !wl) return -1;
    const double* vin[3] = {ut, vt, wt};
    double* vout[3] = {ul, vl, wl};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i)
                for (int a = 0; a < 3; ++a) {
                    int L[3] = {i, j, k}, R[3] = {i, j, k};
                    R[a] += 1;
                    int64_t q = lin(p, i, j, k);
                    if (is_wall_face(p, a, L[a])) {
                        vout[a][q] = 0.0;
                        continue;
                    }
                    double U = vin[a][q];
                    double up = dmin(1.0, dmin(cellv(p, bdn, L), cellv(p, bup, R)));
                    double dn = dmin(1.0, dmin(cellv(p, bup, L), cellv(p, bdn, R)));
                    vout[a][q] = (pos(U) * up) + (neg(U) * dn);
                }
    return 0;
}

/* ------------------------------------------------------------------ */
/* C6: the step                                                       */
/* ------------------------------------------------------------------ */

int ref_step(const ref_problem* p, const double* psin, double* psout,
             const double* cx, const double* cy, const double* cz,
             const double* g)
{
    if (!valid(p) || !psin || !psout || !cx || !cy || !g || psin == psout) return -1;
    int64_t n = ncells(p);
    size_t bytes = sizeof(double) * (size_t)n;
    double* zero = NULL;
    if (!cz) {
        zero = (double*)calloc((size_t)n, sizeof(double));
        if (!zero) return -1;
        cz = zero;
    }
    /* phi (current iterate), next iterate, velocities of the previous pass,
     * antidiffusive velocities, bounds and beta */
    enum { NBUF = 12 };
    double* buf[NBUF];
    for (int b = 0; b < NBUF; ++b) {
        buf[b] = (double*)malloc(bytes);
        if (!buf[b]) {
            for (int c = 0; c < b; ++c) free(buf[c]);
            free(zero);
            return -1;
        }
    }
    double *phi = buf[0], *nxt = buf[1];
    double *pu = buf[2], *pv = buf[3], *pw = buf[4];
    double *au = buf[5], *av = buf[6], *aw = buf[7];
    double *mx = buf[8], *mn = buf[9], *bup = buf[10], *bdn = buf[11];

    /* pass 1: donor cell with the advective Courant numbers */
    ref_donor(p, psin, cx, cy, cz, g, phi);
    memcpy(pu, cx, bytes);
    memcpy(pv, cy, bytes);
    memcpy(pw, cz, bytes);

    for (int m = 2; m <= p->iters; ++m) {
        /* antidiffusive velocities from the current iterate and the
         * previous pass's velocities */
        ref_antidiff(p, phi, pu, pv, pw, g, au, av, aw);
        if (p->limiter) {
            /* bounds from psi^n and the current iterate, then beta; the
             * limited velocities become the next pass's "previous" ones */
            ref_bounds(p, psin, phi, mx, mn);
            ref_beta(p, phi, au, av, aw, mx, mn, g, bup, bdn);
            ref_limit(p, au, av, aw, bup, bdn, pu, pv, pw);
        } else {
            memcpy(pu, au, bytes);
            memcpy(pv, av, bytes);
            memcpy(pw, aw, bytes);
        }
        /* the corrective donor pass on phi with the (limited) velocities */
        ref_donor(p, phi, pu, pv, pw, g, nxt);
        double* t = phi;
        phi = nxt;
        nxt = t;
    }
    memcpy(psout, phi, bytes);
    for (int b = 0; b < NBUF; ++b) free(buf[b]);
    free(zero);
    return 0;
}

int ref_run(const ref_problem* p, int32_t nsteps, double* psi,
            const double* cx, const double* cy, const double* cz,
            const double* g)
{
    if (!valid(p) || nsteps < 0 || !psi) return -1;
    if (nsteps == 0) return 0;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)ncells(p));
    if (!tmp) return -1;
    for (int s = 0; s < nsteps; ++s) {
        int rc = ref_step(p, psi, tmp, cx, cy, cz, g);
        if (rc) {
            free(tmp);
            return rc;
        }
        memcpy(psi, tmp, sizeof(double) * (size_t)ncells(p));
    }
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* C7: mass                                                           */
/* ------------------------------------------------------------------ */

int ref_mass(const ref_problem* p, const double* psi, const double* g, double* out)
{
    if (!valid(p) || !psi || !g || !out) return -1;
    /* Neumaier: running sum s and compensation c, serial in index order */
    double s = 0.0, c = 0.0;
    int64_t n = ncells(p);
    for (int64_t q = 0; q < n; ++q) {
        double x = g[q] * psi[q];
        double t = s + x;
        if (fabs(s) >= fabs(x))
            c += (s - t) + x;
        else
            c += (x - t) + s;
        s = t;
    }
    *out = s + c;
    return 0;
}

int ref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Reverse (adjoint) sweep                                            */
/*                                                                    */
/* Each stage's adjoint is a scatter loop: every forward output       */
/* distributes lam(output) * d(output)/d(input) to the inputs it      */
/* read, through the same halo rules the forward stage used.  At the  */
/* kinks the derivative follows the branch taken:                     */
/*   [c]+ and [c]- have derivatives [c > 0] and [c < 0], and 1/2     */
/*   each at c = 0; |c| has sign(c) with sign(0) = 0;                 */
/*   min(1, min(a, b)) routes to the first minimal entry of (1, a, b) */
/*   (nothing when it is the constant 1);                             */
/*   the bounds route to the first extremal entry of the list         */
/*   psi^n at (self, -x, +x, -y, +y, -z, +z), then phi in the same    */
/*   order.                                                           */
/* ------------------------------------------------------------------ */

/* Linear index of a cell after the halo rule. */
static int64_t cell_lin(const ref_problem* p, const int c[3])
{
    return lin(p, cell_index(p, 0, c[0]), cell_index(p, 1, c[1]), cell_index(p, 2, c[2]));
}

/* Linear index of face c[axis]+1/2 (the same rule as facev), or -1 where the
 * face is a closed wall (the value read there is the constant 0). */
static int64_t face_lin(const ref_problem* p, int axis, const int c[3])
{
    int d[3];
    for (int b = 0; b < 3; ++b)
        d[b] = (b == axis) ? c[b] : cell_index(p, b, c[b]);
    int n = extent(p, axis);
    if (p->bc[axis] == REF_CLOSED) {
        if (d[axis] <= -1 || d[axis] >= n - 1) return -1;
    } else {
        d[axis] = ((d[axis] % n) + n) % n;
    }
    return lin(p, d[0], d[1], d[2]);
}

/* d[c]+/dc and d[c]-/dc.  At c = 0 exactly both are 1/2, the symmetric
 * subgradient: a donor flux [c]+ pL + [c]- pR then has slope (pL + pR)/2,
 * its true derivative whenever pL == pR (which is common: an exactly uniform
 * region gives exactly zero antidiffusive velocities). */
static double step_fn(double c) { return c > 0.0 ? 1.0 : (c < 0.0 ? 0.0 : 0.5); }
static double stepn_fn(double c) { return c < 0.0 ? 1.0 : (c > 0.0 ? 0.0 : 0.5); }
static double sgn(double c) { return c > 0.0 ? 1.0 : (c < 0.0 ? -1.0 : 0.0); }

/* Adjoint of ref_donor: lout -> lphi (+=), lvel[a] (+=). */
static void adj_donor(const ref_problem* p, const double* phi, const double* const vel[3],
                      const double* g, const double* lout, double* lphi, double* const lvel[3])
{
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int c[3] = {i, j, k};
                int64_t q = lin(p, i, j, k);
                lphi[q] += lout[q];   /* out = phi - div / G */
                for (int a = 0; a < 3; ++a) {
                    int64_t fi = face_lin(p, a, c);
                    if (fi < 0) continue;          /* wall: the flux is the constant 0 */
                    int r[3] = {i, j, k};
                    r[a] += 1;
                    int64_t qr = cell_lin(p, r);
                    /* the flux through face c+1/2 leaves c and enters r */
                    double lamf = lout[qr] / g[qr] - lout[q] / g[q];
                    double v = vel[a][fi];
                    lphi[q] += pos(v) * lamf;
                    lphi[qr] += neg(v) * lamf;
                    lvel[a][fi] += (step_fn(v) * phi[q] + stepn_fn(v) * phi[qr]) * lamf;
                }
            }
}

/* Index (0, 1 or 2) of the first minimal entry of (1, x, y). */
static int first_min3(double x, double y)
{
    double m = dmin(1.0, dmin(x, y));
    if (1.0 == m) return 0;
    if (x == m) return 1;
    return 2;
}

/* Adjoint of ref_limit: lvl -> lut (+=), lbup (+=), lbdn (+=). */
static void adj_limit(const ref_problem* p, const double* const ut[3], const double* bup,
                      const double* bdn, const double* const lvl[3], double* const lut[3],
                      double* lbup, double* lbdn)
{
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i)
                for (int a = 0; a < 3; ++a) {
                    int L[3] = {i, j, k}, R[3] = {i, j, k};
                    R[a] += 1;
                    int64_t q = lin(p, i, j, k);
                    if (is_wall_face(p, a, L[a])) continue;
                    int64_t qr = cell_lin(p, R);
                    double U = ut[a][q];
                    double lam = lvl[a][q];
                    double up = dmin(1.0, dmin(bdn[q], bup[qr]));
                    double dn = dmin(1.0, dmin(bup[q], bdn[qr]));
                    lut[a][q] += lam * (step_fn(U) * up + stepn_fn(U) * dn);
                    if (U > 0.0) {
                        int w = first_min3(bdn[q], bup[qr]);
                        if (w == 1) lbdn[q] += lam * U;
                        if (w == 2) lbup[qr] += lam * U;
                    } else if (U < 0.0) {
                        int w = first_min3(bup[q], bdn[qr]);
                        if (w == 1) lbup[q] += lam * U;
                        if (w == 2) lbdn[qr] += lam * U;
                    }
                }
}

/* Adjoint of ref_beta: (lbup, lbdn) -> lphi (+=), lut (+=), lmx (+=), lmn (+=). */
static void adj_beta(const ref_problem* p, const double* phi, const double* const ut[3],
                     const double* mx, const double* mn, const double* g, const double* lbup,
                     const double* lbdn, double* lphi, double* const lut[3], double* lmx, double* lmn)
{
    const double eps = eps_of(p);
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int c[3] = {i, j, k};
                int64_t q = lin(p, i, j, k);
                /* recompute in and out as ref_beta does */
                double fin[3], fout[3];
                int64_t fl[3], fr[3], ql[3], qr[3];
                double vl[3], vr[3];
                for (int a = 0; a < 3; ++a) {
                    int l[3] = {i, j, k}, r[3] = {i, j, k};
                    l[a] -= 1;
                    r[a] += 1;
                    fr[a] = face_lin(p, a, c);
                    fl[a] = face_lin(p, a, l);
                    vr[a] = fr[a] < 0 ? 0.0 : ut[a][fr[a]];
                    vl[a] = fl[a] < 0 ? 0.0 : ut[a][fl[a]];
                    ql[a] = cell_lin(p, l);
                    qr[a] = cell_lin(p, r);
                    fin[a] = pos(vl[a]) * phi[ql[a]] - neg(vr[a]) * phi[qr[a]];
                    fout[a] = pos(vr[a]) * phi[q] - neg(vl[a]) * phi[q];
                }
                double in = ((fin[0] + fin[1]) + fin[2]);
                double out = ((fout[0] + fout[1]) + fout[2]);
                double din = in + eps, dout = out + eps;
                double bu = ((mx[q] - phi[q]) * g[q]) / din;
                double bd = ((phi[q] - mn[q]) * g[q]) / dout;
                double gu = lbup[q], gd = lbdn[q];
                lmx[q] += gu * g[q] / din;
                lmn[q] -= gd * g[q] / dout;
                lphi[q] += -gu * g[q] / din + gd * g[q] / dout;
                double lin_ = -gu * bu / din;
                double lout_ = -gd * bd / dout;
                for (int a = 0; a < 3; ++a) {
                    /* in = sum [vl]+ phi(l) - [vr]- phi(r) */
                    lphi[ql[a]] += lin_ * pos(vl[a]);
                    lphi[qr[a]] -= lin_ * neg(vr[a]);
                    if (fl[a] >= 0) lut[a][fl[a]] += lin_ * step_fn(vl[a]) * phi[ql[a]];
                    if (fr[a] >= 0) lut[a][fr[a]] -= lin_ * stepn_fn(vr[a]) * phi[qr[a]];
                    /* out = sum [vr]+ phi(c) - [vl]- phi(c) */
                    lphi[q] += lout_ * (pos(vr[a]) - neg(vl[a]));
                    if (fr[a] >= 0) lut[a][fr[a]] += lout_ * step_fn(vr[a]) * phi[q];
                    if (fl[a] >= 0) lut[a][fl[a]] -= lout_ * stepn_fn(vl[a]) * phi[q];
                }
            }
}

/* Adjoint of ref_bounds: (lmx, lmn) -> lpsin (+=), lphi (+=). */
static void adj_bounds(const ref_problem* p, const double* psin, const double* phi, const double* lmx,
                       const double* lmn, double* lpsin, double* lphi)
{
    static const int off[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                int64_t q = lin(p, i, j, k);
                int64_t idx[14];
                double val[14];
                for (int f = 0; f < 2; ++f)
                    for (int o = 0; o < 7; ++o) {
                        int d[3] = {i + off[o][0], j + off[o][1], k + off[o][2]};
                        idx[f * 7 + o] = cell_lin(p, d);
                        val[f * 7 + o] = (f == 0 ? psin : phi)[idx[f * 7 + o]];
                    }
                int am = 0, an = 0;
                for (int e = 1; e < 14; ++e) {
                    if (val[e] > val[am]) am = e;
                    if (val[e] < val[an]) an = e;
                }
                (am < 7 ? lpsin : lphi)[idx[am]] += lmx[q];
                (an < 7 ? lpsin : lphi)[idx[an]] += lmn[q];
            }
}

/* Adjoint of ref_antidiff: lut -> lphi (+=), lvel (+=). */
static void adj_antidiff(const ref_problem* p, const double* phi, const double* const vel[3],
                         const double* g, const double* const lut[3], double* lphi, double* const lvel[3])
{
    const double eps = eps_of(p);
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i)
                for (int a = 0; a < 3; ++a) {
                    int L[3] = {i, j, k};
                    int64_t q = lin(p, i, j, k);
                    if (is_wall_face(p, a, L[a])) continue;
                    double lam = lut[a][q];
                    int R[3] = {i, j, k};
                    R[a] += 1;
                    int tr[2], nt = 0;
                    for (int b = 0; b < 3; ++b)
                        if (b != a) tr[nt++] = b;
                    int64_t qL = cell_lin(p, L), qR = cell_lin(p, R);
                    double pL = phi[qL], pR = phi[qR];
                    double D0 = (pR + pL) + eps;
                    double A = (pR - pL) / D0;
                    double B[2], Vb[2], Dt[2], Sp[2], Sm[2];
                    int64_t qLp[2], qRp[2], qLm[2], qRm[2], f4[2][4];
                    for (int s = 0; s < 2; ++s) {
                        int t = tr[s];
                        int Lp[3] = {L[0], L[1], L[2]}, Rp[3] = {R[0], R[1], R[2]};
                        int Lm[3] = {L[0], L[1], L[2]}, Rm[3] = {R[0], R[1], R[2]};
                        Lp[t] += 1; Rp[t] += 1; Lm[t] -= 1; Rm[t] -= 1;
                        qLp[s] = cell_lin(p, Lp); qRp[s] = cell_lin(p, Rp);
                        qLm[s] = cell_lin(p, Lm); qRm[s] = cell_lin(p, Rm);
                        Sp[s] = phi[qRp[s]] + phi[qLp[s]];
                        Sm[s] = phi[qRm[s]] + phi[qLm[s]];
                        Dt[s] = (Sp[s] + Sm[s]) + eps;
                        B[s] = 0.5 * ((Sp[s] - Sm[s]) / Dt[s]);
                        f4[s][0] = face_lin(p, t, L);
                        f4[s][1] = face_lin(p, t, R);
                        f4[s][2] = face_lin(p, t, Lm);
                        f4[s][3] = face_lin(p, t, Rm);
                        double vs = 0.0;
                        double fv[4];
                        for (int e = 0; e < 4; ++e) fv[e] = f4[s][e] < 0 ? 0.0 : vel[t][f4[s][e]];
                        vs = (fv[0] + fv[1]) + (fv[2] + fv[3]);
                        Vb[s] = 0.25 * vs;
                    }
                    double Gf = 0.5 * (g[qL] + g[qR]);
                    double U = vel[a][q];
                    double S = (Vb[0] * B[0]) + (Vb[1] * B[1]);
                    /* U~ = (|U| - U^2/Gf) A - (U/Gf) S */
                    double dU = (sgn(U) - 2.0 * U / Gf) * A - S / Gf;
                    double dA = fabs(U) - (U * U) / Gf;
                    double dS = -U / Gf;
                    lvel[a][q] += lam * dU;
                    double gA = lam * dA;
                    lphi[qR] += gA * (2.0 * pL + eps) / (D0 * D0);
                    lphi[qL] -= gA * (2.0 * pR + eps) / (D0 * D0);
                    for (int s = 0; s < 2; ++s) {
                        double gB = lam * dS * Vb[s];
                        double gV = lam * dS * B[s];
                        double dSp = 0.5 * (2.0 * Sm[s] + eps) / (Dt[s] * Dt[s]);
                        double dSm = -0.5 * (2.0 * Sp[s] + eps) / (Dt[s] * Dt[s]);
                        lphi[qRp[s]] += gB * dSp;
                        lphi[qLp[s]] += gB * dSp;
                        lphi[qRm[s]] += gB * dSm;
                        lphi[qLm[s]] += gB * dSm;
                        for (int e = 0; e < 4; ++e)
                            if (f4[s][e] >= 0) lvel[tr[s]][f4[s][e]] += 0.25 * gV;
                    }
                }
}

int ref_adjoint(const ref_problem* p, int32_t nsteps, const double* psi0,
                const double* cx, const double* cy, const double* cz,
                const double* g, const double* seed, double* dpsi0,
                double* dcx, double* dcy, double* dcz)
{
    if (!valid(p) || nsteps < 0 || !psi0 || !cx || !cy || !g || !seed || !dpsi0 || !dcx || !dcy) return -1;
    const int64_t n = ncells(p);
    const size_t bytes = sizeof(double) * (size_t)n;
    const int M = p->iters;
    double* zero = (double*)calloc((size_t)n, sizeof(double));
    double* dcz_local = (double*)calloc((size_t)n, sizeof(double));
    /* states psi^0..psi^{nsteps-1}; per pass m: phi_m, U~_m (3), V_m (3), mx, mn, bup, bdn */
    double* states = (double*)malloc(bytes * (size_t)(nsteps > 0 ? nsteps : 1));
    double* phis = (double*)malloc(bytes * (size_t)(M + 1));
    double* uts = (double*)malloc(bytes * 3 * (size_t)(M + 1));
    double* vls = (double*)malloc(bytes * 3 * (size_t)(M + 1));
    double* bnd = (double*)malloc(bytes * 4 * (size_t)(M + 1));
    double* lam = (double*)malloc(bytes * 12);
    if (!zero || !dcz_local || !states || !phis || !uts || !vls || !bnd || !lam) {
        free(zero); free(dcz_local); free(states); free(phis); free(uts); free(vls); free(bnd); free(lam);
        return -1;
    }
    if (!cz) cz = zero;
    double* dC[3] = {dcx, dcy, dcz ? dcz : dcz_local};
    memset(dcx, 0, bytes);
    memset(dcy, 0, bytes);
    memset(dC[2], 0, bytes);

    /* forward sweep storing the step states */
    if (nsteps > 0) memcpy(states, psi0, bytes);
    for (int s = 1; s < nsteps; ++s)
        ref_step(p, states + (size_t)(s - 1) * n, states + (size_t)s * n, cx, cy, cz, g);

    double* lcur = lam;              /* adjoint of the current iterate  */
    double* lprev = lam + n;         /* adjoint of the previous iterate */
    double* lpsin = lam + 2 * n;     /* adjoint of psi^n                */
    double* lv[3] = {lam + 3 * n, lam + 4 * n, lam + 5 * n};     /* of V_m     */
    double* lvp[3] = {lam + 6 * n, lam + 7 * n, lam + 8 * n};    /* of V_{m-1} */
    double* lb = lam + 9 * n;        /* of beta_up, beta_dn (2 fields)  */
    double* lmxmn = lam + 11 * n;    /* of mx (lmn reuses lb after beta) */
    double* lut_[3] = {NULL, NULL, NULL};
    double* lutbuf = (double*)malloc(bytes * 5);
    if (!lutbuf) {
        free(zero); free(dcz_local); free(states); free(phis); free(uts); free(vls); free(bnd); free(lam);
        return -1;
    }
    double* lmn = lutbuf + 3 * n;
    double* lbdn = lutbuf + 4 * n;
    for (int a = 0; a < 3; ++a) lut_[a] = lutbuf + (size_t)a * n;

    memcpy(lcur, seed, bytes);
    const double* C3[3] = {cx, cy, cz};
    for (int s = nsteps - 1; s >= 0; --s) {
        const double* psin = states + (size_t)s * n;
        /* recompute the step's intermediates, pass by pass */
        ref_donor(p, psin, cx, cy, cz, g, phis + (size_t)1 * n);
        for (int m = 2; m <= M; ++m) {
            const double* prev[3];
            for (int a = 0; a < 3; ++a)
                prev[a] = (m == 2) ? C3[a] : vls + ((size_t)3 * (m - 1) + a) * n;
            double* U3[3] = {uts + ((size_t)3 * m) * n, uts + ((size_t)3 * m + 1) * n, uts + ((size_t)3 * m + 2) * n};
            double* V3[3] = {vls + ((size_t)3 * m) * n, vls + ((size_t)3 * m + 1) * n, vls + ((size_t)3 * m + 2) * n};
            double* B4 = bnd + (size_t)4 * m * n;
            const double* ph = phis + (size_t)(m - 1) * n;
            ref_antidiff(p, ph, prev[0], prev[1], prev[2], g, U3[0], U3[1], U3[2]);
            if (p->limiter) {
                ref_bounds(p, psin, ph, B4, B4 + n);
                ref_beta(p, ph, U3[0], U3[1], U3[2], B4, B4 + n, g, B4 + 2 * n, B4 + 3 * n);
                ref_limit(p, U3[0], U3[1], U3[2], B4 + 2 * n, B4 + 3 * n, V3[0], V3[1], V3[2]);
            } else {
                for (int a = 0; a < 3; ++a) memcpy(V3[a], U3[a], bytes);
            }
            ref_donor(p, ph, V3[0], V3[1], V3[2], g, phis + (size_t)m * n);
        }

        /* reverse through the passes */
        memset(lpsin, 0, bytes);
        for (int a = 0; a < 3; ++a) memset(lv[a], 0, bytes);
        for (int m = M; m >= 2; --m) {
            const double* ph = phis + (size_t)(m - 1) * n;
            const double* V3[3] = {vls + ((size_t)3 * m) * n, vls + ((size_t)3 * m + 1) * n, vls + ((size_t)3 * m + 2) * n};
            const double* U3[3] = {uts + ((size_t)3 * m) * n, uts + ((size_t)3 * m + 1) * n, uts + ((size_t)3 * m + 2) * n};
            const double* B4 = bnd + (size_t)4 * m * n;
            const double* prev[3];
            for (int a = 0; a < 3; ++a)
                prev[a] = (m == 2) ? C3[a] : vls + ((size_t)3 * (m - 1) + a) * n;
            memset(lprev, 0, bytes);
            for (int a = 0; a < 3; ++a) memset(lvp[a], 0, bytes);
            /* phi_m = donor(phi_{m-1}, V_m): lv already holds the A-adjoint part from pass m+1 */
            adj_donor(p, ph, V3, g, lcur, lprev, lv);
            if (p->limiter) {
                for (int a = 0; a < 3; ++a) memset(lut_[a], 0, bytes);
                memset(lb, 0, bytes);
                memset(lbdn, 0, bytes);
                memset(lmxmn, 0, bytes);
                memset(lmn, 0, bytes);
                adj_limit(p, U3, B4 + 2 * n, B4 + 3 * n, (const double* const*)lv, lut_, lb, lbdn);
                adj_beta(p, ph, U3, B4, B4 + n, g, lb, lbdn, lprev, lut_, lmxmn, lmn);
                adj_bounds(p, psin, ph, lmxmn, lmn, lpsin, lprev);
            } else {
                for (int a = 0; a < 3; ++a) memcpy(lut_[a], lv[a], bytes);
            }
            double* const* lvtarget = (m == 2) ? dC : lvp;
            adj_antidiff(p, ph, prev, g, (const double* const*)lut_, lprev, lvtarget);
            /* move to pass m-1 */
            double* t = lcur;
            lcur = lprev;
            lprev = t;
            for (int a = 0; a < 3; ++a) {
                double* tt = lv[a];
                lv[a] = lvp[a];
                lvp[a] = tt;
            }
        }
        /* pass 1: phi_1 = donor(psi^n, C) */
        adj_donor(p, psin, C3, g, lcur, lpsin, dC);
        memcpy(lcur, lpsin, bytes);
    }
    memcpy(dpsi0, lcur, bytes);
    free(lutbuf); free(zero); free(dcz_local); free(states); free(phis); free(uts); free(vls); free(bnd); free(lam);
    return 0;
}


/* ------------------------------------------------------------------------
 * Unstructured (edge-based) donor-cell step, the paper's operator sequence
 * (Listing 8): upwind edge fluxes, vertical fluxes, divergence, update.
 * ------------------------------------------------------------------------ */
int ref_ustep(const ref_umesh* m, const int32_t* edges, const int32_t* node_ptr, const int32_t* node_edges,
              const int8_t* node_sign, const double* vol, const double* psi, const double* vn,
              const double* w, const double* rho, double* out)
{
    if (!m || m->n_nodes < 1 || m->n_edges < 0 || m->nz < 1 || !edges || !node_ptr || !node_edges ||
        !node_sign || !vol || !psi || !vn || !w || !rho || !out)
        return -1;
    const int64_t nn = m->n_nodes, ne = m->n_edges, nz = m->nz;
    if (node_ptr[0] != 0 || node_ptr[nn] != 2 * ne) return -1;
    for (int64_t n = 0; n < nn; ++n)
        if (node_ptr[n + 1] < node_ptr[n]) return -1;
    for (int64_t n = 0; n < nn; ++n)
        if (!(vol[n] > 0.0)) return -1;
    for (int64_t e = 0; e < 2 * ne; ++e)
        if (edges[e] < 0 || edges[e] >= nn) return -1;
    for (int64_t j = 0; j < 2 * ne; ++j)
        if (node_edges[j] < 0 || node_edges[j] >= ne || (node_sign[j] != 1 && node_sign[j] != -1)) return -1;

    double* flux = malloc(sizeof(double) * (size_t)(ne > 0 ? ne * nz : 1));
    double* fz = malloc(sizeof(double) * (size_t)(nn * (nz + 1)));
    if (!flux || !fz) {
        free(flux);
        free(fz);
        return -1;
    }
    /* upwind flux on the edges (Listings 4-5) */
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t a = edges[2 * e], b = edges[2 * e + 1];
        for (int64_t k = 0; k < nz; ++k) {
            const double v = vn[e * nz + k];
            flux[e * nz + k] = pos(v) * psi[a * nz + k] + neg(v) * psi[b * nz + k];
        }
    }
    /* vertical upwind flux at the level interfaces (Listing 7) */
    for (int64_t n = 0; n < nn; ++n) {
        double* f = fz + n * (nz + 1);
        const double* p = psi + n * nz;
        const double* wn = w + n * nz;
        if (nz == 1) {
            f[0] = f[1] = 0.0;
            continue;
        }
        for (int64_t k = 1; k < nz; ++k) f[k] = pos(wn[k]) * p[k - 1] + neg(wn[k]) * p[k];
        f[0] = m->pivbz * f[1];
        f[nz] = m->pivbz * f[nz - 1];
    }
    /* flux divergence over the dual volume and the update (Listing 8) */
    for (int64_t n = 0; n < nn; ++n)
        for (int64_t k = 0; k < nz; ++k) {
            double acc = 0.0;
            for (int32_t j = node_ptr[n]; j < node_ptr[n + 1]; ++j)
                acc += (double)node_sign[j] * flux[(int64_t)node_edges[j] * nz + k];
            const double div = acc / vol[n] + (fz[n * (nz + 1) + k + 1] - fz[n * (nz + 1) + k]);
            out[n * nz + k] = psi[n * nz + k] - div / rho[n * nz + k];
        }
    free(flux);
    free(fz);
    return 0;
}
