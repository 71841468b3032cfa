/*
 * mpdata_ref.h -- CPU FP64 oracle for one MPDATA time step on a 3-D
 * structured grid.  TEST INFRASTRUCTURE ONLY: the GPU library never includes,
 * links or calls anything declared here, and this oracle shares no code with
 * it.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * use it.
 *
 * The scheme: a donor-cell (upwind) pass, the paper's upwind flux, vertical
 * flux, flux divergence and solution update (Section 5, Listings 4-9),
 * followed by (iters-1) antidiffusive corrective passes, each optionally
 * limited by the non-oscillatory (flux-corrected transport) limiter.  The
 * paper shows only the upwind stages and refers to another project
 * deliverable for the rest (Section 5); the corrective passes are written
 * here from the published scheme (Smolarkiewicz 1984; Smolarkiewicz & Grabowski 1990;
 * Smolarkiewicz & Margolin 1998) in the metric (G-weighted) flux form
 *     d(G psi)/dt + div(V psi) = 0,   C = dt V / dx on staggered faces.
 *
 * Layout: every field is dense C order [nz][ny][nx], i fastest.  Face arrays
 * share the cell index space (Section 3.1.4.1, the C-grid convention): cx[k][j][i]
 * is the Courant number on the face (i+1/2, j, k), cy on (i, j+1/2, k) and
 * cz on (i, j, k+1/2).  On a periodic axis the last slot is the wrap face
 * n-1/2 == -1/2; on a closed axis the faces -1/2 and n-1/2 carry no flux and
 * the slot n-1 is never read.
 *
 * Arithmetic: IEEE FP64, no contraction, evaluated exactly as parenthesised
 * in mpdata_ref.c.  All pointers are host pointers.  Functions return 0 on
 * success and -1 on an invalid argument (nothing is written then).
 */
#ifndef MPDATA_REF_H
#define MPDATA_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_PERIODIC = 0, REF_CLOSED = 1 };

typedef struct {
    int32_t nx, ny, nz;   /* cells per axis, each >= 1                       */
    int32_t bc[3];        /* per axis x, y, z: REF_PERIODIC or REF_CLOSED     */
    int32_t iters;        /* passes per step, >= 1 (1 = donor cell only)      */
    int32_t limiter;      /* 0 = off, 1 = non-oscillatory limiter             */
    double eps;           /* denominator guard; 0 selects 1e-15               */
} ref_problem;

/* Donor-cell pass on phi with face velocities (u, v, w): out = phi - div/G. */
int ref_donor(const ref_problem* p, const double* phi, const double* u,
              const double* v, const double* w, const double* g, double* out);

/* Antidiffusive pseudo-velocities from the iterate phi and the previous
 * pass's velocities (u, v, w); zero on closed-boundary faces. */
int ref_antidiff(const ref_problem* p, const double* phi, const double* u,
                 const double* v, const double* w, const double* g,
                 double* ut, double* vt, double* wt);

/* Local bounds: max / min over the 7-point neighbourhood of psin and phi. */
int ref_bounds(const ref_problem* p, const double* psin, const double* phi,
               double* mx, double* mn);

/* Limiter coefficients beta_up (inflow) and beta_dn (outflow). */
int ref_beta(const ref_problem* p, const double* phi, const double* ut,
             const double* vt, const double* wt, const double* mx,
             const double* mn, const double* g, double* bup, double* bdn);

/* Limited velocities from (ut, vt, wt) and the two beta fields. */
int ref_limit(const ref_problem* p, const double* ut, const double* vt,
              const double* wt, const double* bup, const double* bdn,
              double* ul, double* vl, double* wl);

/* One full step psin -> psout (distinct arrays).  cz may be NULL (all 0). */
int ref_step(const ref_problem* p, const double* psin, double* psout,
             const double* cx, const double* cy, const double* cz,
             const double* g);

/* nsteps steps in place on psi. */
int ref_run(const ref_problem* p, int32_t nsteps, double* psi,
            const double* cx, const double* cy, const double* cz,
            const double* g);

/* Mass sum(G * psi) with Neumaier compensated summation. */
int ref_mass(const ref_problem* p, const double* psi, const double* g,
             double* out);

/* Reverse (adjoint) sweep of ref_run.  Given the seed lam = dJ/dpsi_T of a
 * cost J(psi_T), returns dJ/dpsi0 and dJ/d(cx, cy, cz) (dcz may be NULL).
 * Every step's intermediates are recomputed from stored step states; at the
 * kinks of max/min the derivative follows the argument taken, the first
 * extremal one in a fixed order, and [c]+- take slope 1/2 at c = 0 (see
 * mpdata_ref.c).  Plain scatter loops,
 * serial. */
int ref_adjoint(const ref_problem* p, int32_t nsteps, const double* psi0,
                const double* cx, const double* cy, const double* cz,
                const double* g, const double* seed, double* dpsi0,
                double* dcx, double* dcy, double* dcz);

/* Threads the oracle's parallel loops use (OpenMP). */
int ref_num_threads(void);
/* Threads of later calls (OpenMP builds; n >= 1). */
void ref_set_num_threads(int n);

/* ------------------------------------------------------------------------
 * Edge-based donor-cell step on an unstructured mesh (the paper's own MPDATA
 * dwarf, Section 5, Listings 4-9): upwind flux on every edge (Listings 4-5),
 * vertical upwind flux with the boundary factor pivbz (Listing 7), flux
 * divergence at the nodes through the node-to-edge table and its signs,
 * divided by the dual volume (Listing 8), and the solution update.
 *
 * Layout: per-node fields (n_nodes, nz), per-edge fields (n_edges, nz),
 * level fastest.  edges[2e], edges[2e+1] = ip1, ip2; a positive vn[e][k]
 * carries psi from ip1 to ip2.  node_edges[node_ptr[n] .. node_ptr[n+1]) are
 * node n's edges with node_sign +1 where n is the edge's ip1, -1 where it is
 * ip2.  w[n][k] (k >= 1) is the vertical Courant number at the interface
 * between levels k-1 and k (w[n][0] is not read).
 *
 *   flux[e][k] = max(0, vn) psi[ip1][k] + min(0, vn) psi[ip2][k]
 *   fz[n][k]   = max(0, w[n][k]) psi[n][k-1] + min(0, w[n][k]) psi[n][k], 1 <= k <= nz-1
 *   fz[n][0]   = pivbz fz[n][1],  fz[n][nz] = pivbz fz[n][nz-1]   (nz = 1: no vertical flux)
 *   div[n][k]  = (sum over n's edges, in table order, of sign * flux) / vol[n]
 *                + (fz[n][k+1] - fz[n][k])
 *   out[n][k]  = psi[n][k] - div[n][k] / rho[n][k]
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_nodes, n_edges, nz;
    double pivbz;
} ref_umesh;

int ref_ustep(const ref_umesh* m, const int32_t* edges, const int32_t* node_ptr, const int32_t* node_edges,
              const int8_t* node_sign, const double* vol, const double* psi, const double* vn,
              const double* w, const double* rho, double* out);

#ifdef __cplusplus
}
#endif
#endif
