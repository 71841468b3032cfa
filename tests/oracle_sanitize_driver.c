/* Drives every entry point of the CPU oracle (oracle/mpdata_ref.c) over
 * small and degenerate grids, every boundary combination and pass count,
 * on heap arrays of exactly the documented sizes, so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer reports any access outside
 * them or any undefined operation.  Test infrastructure: built and run by
 * tests/test_oracle_sanitized.py.  Exits 0 when every call returned 0 and
 * every output is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "mpdata_ref.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

/* splitmix64 (Steele, Lea and Flood), mapped to [0, 1) */
static double uniform01(void)
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static double* field(size_t n, double lo, double hi)
{
    double* a = malloc(n * sizeof(double));
    if (!a) exit(3);
    for (size_t i = 0; i < n; ++i) a[i] = lo + (hi - lo) * uniform01();
    return a;
}

static int finite_all(const double* a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int failures = 0;

static void check(int ok, const char* what, int nx, int ny, int nz)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s on %dx%dx%d\n", what, nx, ny, nz);
        ++failures;
    }
}

static void structured(int nx, int ny, int nz, int bx, int by, int bz, int iters, int limiter, double eps)
{
    const size_t n = (size_t)nx * ny * nz;
    ref_problem p = {nx, ny, nz, {bx, by, bz}, iters, limiter, eps};
    double* psi = field(n, 0.0, 1.0);
    double* g = field(n, 0.5, 1.0);
    double* cx = field(n, -0.05, 0.05);
    double* cy = field(n, -0.05, 0.05);
    double* cz = field(n, -0.05, 0.05);
    double* out = field(n, 0.0, 0.0);
    double* a[9];
    for (int i = 0; i < 9; ++i) a[i] = field(n, 0.0, 0.0);
    if (n > 2) psi[n / 2] = 0.0;   /* an exact zero */

    check(ref_donor(&p, psi, cx, cy, cz, g, out) == 0 && finite_all(out, n), "ref_donor", nx, ny, nz);
    check(ref_antidiff(&p, psi, cx, cy, cz, g, a[0], a[1], a[2]) == 0 && finite_all(a[0], n), "ref_antidiff", nx,
          ny, nz);
    check(ref_bounds(&p, psi, out, a[3], a[4]) == 0, "ref_bounds", nx, ny, nz);
    check(ref_beta(&p, out, a[0], a[1], a[2], a[3], a[4], g, a[5], a[6]) == 0 && finite_all(a[5], n), "ref_beta",
          nx, ny, nz);
    check(ref_limit(&p, a[0], a[1], a[2], a[5], a[6], a[7], a[8], out) == 0 && finite_all(a[7], n), "ref_limit",
          nx, ny, nz);
    check(ref_step(&p, psi, out, cx, cy, cz, g) == 0 && finite_all(out, n), "ref_step", nx, ny, nz);
    check(ref_step(&p, psi, out, cx, cy, NULL, g) == 0 && finite_all(out, n), "ref_step (cz NULL)", nx, ny, nz);
    check(ref_run(&p, 3, psi, cx, cy, cz, g) == 0 && finite_all(psi, n), "ref_run", nx, ny, nz);
    double m = 0.0;
    check(ref_mass(&p, psi, g, &m) == 0 && isfinite(m), "ref_mass", nx, ny, nz);
    for (size_t i = 0; i < n; ++i) a[0][i] = 2.0 * psi[i];
    check(ref_adjoint(&p, 3, psi, cx, cy, cz, g, a[0], a[1], a[2], a[3], a[4]) == 0 && finite_all(a[1], n) &&
              finite_all(a[2], n) && finite_all(a[4], n),
          "ref_adjoint", nx, ny, nz);
    check(ref_adjoint(&p, 2, psi, cx, cy, NULL, g, a[0], a[1], a[2], a[3], NULL) == 0 && finite_all(a[1], n),
          "ref_adjoint (cz NULL)", nx, ny, nz);

    free(psi); free(g); free(cx); free(cy); free(cz); free(out);
    for (int i = 0; i < 9; ++i) free(a[i]);
}

/* A ring of `nn` nodes (edge e joins node e and e+1 mod nn), nz levels. */
static void ring(int nn, int nz, double pivbz, int with_w)
{
    const int ne = nn;
    int32_t* edges = malloc(sizeof(int32_t) * 2 * ne);
    int32_t* ptr = malloc(sizeof(int32_t) * (nn + 1));
    int32_t* ned = malloc(sizeof(int32_t) * 2 * ne);
    int8_t* sgn = malloc(2 * ne);
    if (!edges || !ptr || !ned || !sgn) exit(3);
    for (int e = 0; e < ne; ++e) {
        edges[2 * e] = e;
        edges[2 * e + 1] = (e + 1) % nn;
    }
    for (int v = 0; v < nn; ++v) {
        ptr[v] = 2 * v;
        ned[2 * v] = (v + nn - 1) % nn;   /* the edge arriving at v: v is its ip2 */
        sgn[2 * v] = -1;
        ned[2 * v + 1] = v;               /* the edge leaving v: v is its ip1 */
        sgn[2 * v + 1] = 1;
    }
    ptr[nn] = 2 * nn;
    const size_t nnodes = (size_t)nn * nz, nedges = (size_t)ne * nz;
    double* vol = field((size_t)nn, 1.0, 2.0);
    double* psi = field(nnodes, 0.0, 1.0);
    double* vn = field(nedges, -0.2, 0.2);
    double* w = with_w ? field(nnodes, -0.2, 0.2) : field(nnodes, 0.0, 0.0);   /* the oracle reads w */
    double* rho = field(nnodes, 1.0, 1.5);
    double* out = field(nnodes, 0.0, 0.0);
    ref_umesh m = {nn, ne, nz, pivbz};
    check(ref_ustep(&m, edges, ptr, ned, sgn, vol, psi, vn, w, rho, out) == 0 && finite_all(out, nnodes),
          "ref_ustep", nn, ne, nz);
    free(edges); free(ptr); free(ned); free(sgn); free(vol); free(psi); free(vn); free(w); free(rho); free(out);
}

int main(void)
{
    const int shapes[][3] = {{1, 1, 1}, {7, 1, 3}, {1, 6, 4}, {2, 2, 3}, {5, 4, 1}, {9, 7, 5}, {3, 2, 12}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (int bc = 0; bc < 8; ++bc)
            for (int iters = 1; iters <= 3; ++iters)
                for (int lim = 0; lim <= 1; ++lim)
                    structured(shapes[s][0], shapes[s][1], shapes[s][2], bc & 1, (bc >> 1) & 1, (bc >> 2) & 1,
                               iters, lim, lim ? 1e-30 : 0.0);
    structured(6, 5, 4, REF_PERIODIC, REF_CLOSED, REF_CLOSED, 8, 1, 0.0);
    ring(3, 1, 0.0, 0);
    ring(5, 4, 0.5, 1);
    ring(8, 3, 1.0, 1);
    if (failures) {
        fprintf(stderr, "%d oracle call(s) failed\n", failures);
        return 1;
    }
    printf("oracle under sanitizers: all calls clean\n");
    return 0;
}
