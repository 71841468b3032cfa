// adjoint.hpp -- reverse-mode (adjoint) kernels of one MPDATA step, FP64.
//
// Every kernel is a gather: one thread owns one cell and writes only that
// cell's adjoint values (and those of its three "own" faces i+1/2, j+1/2,
// k+1/2), collecting lambda(output) * d(output)/d(input) from every forward
// output that read the input.  No atomics, so the adjoint is bitwise
// reproducible.  The stage formulas are those of stages.hpp (the donor-cell
// update of the paper's Listing 8 stages, the antidiffusive velocity, the
// limiter bounds, beta and the limited velocities).  At kinks the derivative
// follows the branch taken: [c]+ has derivative [c > 0], [c]- has [c < 0],
// each 1/2 at c = 0; |c| has sign(c) with sign(0) = 0; min(1, min(a, b)) routes to the first
// minimal entry of (1, a, b); the bounds route to the first extremal entry of
// psi^n at (self, -x, +x, -y, +y, -z, +z), then phi in the same order.
//
// The antidiffusive velocity reads ~20 inputs per face, so its adjoint runs
// in two kernels: the first evaluates each face's partial derivatives times
// the face's adjoint once (seven values per face kept, two applied at
// once), the second gathers them.  In a limited pass the donor-cell adjoint
// and the limiter's run in two kernels: the donor-cell terms with the
// limited velocities' and beta's per-cell terms (k_adj_donor_limit_beta),
// then the gathers of in / out and of the bounds together with the first
// antidiffusive-velocity kernel (k_adj_inout_bounds_antidiff1).  An
// unlimited pass and the first (donor-cell) pass use k_adj_donor, and an
// unlimited pass k_adj_antidiff1 on its own.
#pragma once

#include "common.hpp"
#include "stages.hpp"

namespace mpdata {
namespace adj {

#pragma clang fp contract(off)

using stages::at;
using stages::Cell;
using stages::cell_of_thread;
using stages::closed;
using stages::extent;

// Linear index of the face c[axis]+1/2 for coordinates within one cell of the
// domain (the coordinate along the axis in [-1, n-1]), or -1 at a closed wall.
__device__ __forceinline__ long long face_idx(const Geo& g, int axis, int i, int j, int k)
{
    int c[3] = {i, j, k};
    const int n = extent(g, axis);
    for (int b = 0; b < 3; ++b)
        if (b != axis) c[b] = nbr(c[b], extent(g, b), closed(g, b));
    int f = c[axis];
    if (closed(g, axis)) {
        if (f < 0 || f >= n - 1) return -1;
    } else if (f < 0) {
        f += n;
    }
    c[axis] = f;
    return (long long)c[2] * g.sz + (long long)c[1] * g.sy + c[0];
}

// d[c]+/dc and d[c]-/dc, each 1/2 at c = 0 (the symmetric subgradient: exact
// for a donor flux whose upwind and downwind values are equal)
__device__ __forceinline__ double stp(double c) { return c > 0.0 ? 1.0 : (c < 0.0 ? 0.0 : 0.5); }
__device__ __forceinline__ double stn(double c) { return c < 0.0 ? 1.0 : (c > 0.0 ? 0.0 : 0.5); }
__device__ __forceinline__ double sgn(double c) { return c > 0.0 ? 1.0 : (c < 0.0 ? -1.0 : 0.0); }
__device__ __forceinline__ double ppos(double c) { return c > 0.0 ? c : 0.0; }
__device__ __forceinline__ double pneg(double c) { return c < 0.0 ? c : 0.0; }

// 1/d from the hardware reciprocal refined by two Newton steps (within an
// ulp of the correctly rounded reciprocal; d is a normal positive number).
// A kernel that divides several values by the same denominator multiplies
// by this instead (an IEEE FP64 division is about ten instructions); the
// partial derivatives then differ from the quotients' by a few ulp.
__device__ __forceinline__ double rcp_nr(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}

// Index (0, 1, 2) of the first minimal entry of (1, x, y).
__device__ __forceinline__ int first_min3(double x, double y)
{
    const double m = min2(1.0, min2(x, y));
    if (1.0 == m) return 0;
    if (x == m) return 1;
    return 2;
}

// ---------------------------------------------------------------------------
// Donor-cell pass out = phi - div(F)/G:  lout -> lphi, lvel (each += or, for
// the first contribution a buffer receives, =; an assigned velocity adjoint
// is 0 at a closed wall's unused slot)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adj_donor(Geo g, const double* __restrict__ phi, const double* __restrict__ u,
                                                   const double* __restrict__ v, const double* __restrict__ w,
                                                   const double* __restrict__ gm, const double* __restrict__ lout,
                                                   double* __restrict__ lphi, double* __restrict__ lu,
                                                   double* __restrict__ lv, double* __restrict__ lw, int assign_phi,
                                                   int assign_vel)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    const double* vel[3] = {u, v, w};
    double* lvel[3] = {lu, lv, lw};
    double acc = lout[c.q];
    const double mu_c = lout[c.q] / gm[c.q];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // own face c+1/2 (its slot is c's): the flux leaves c and enters r
        long long fo = face_idx(g, a, c.i, c.j, c.k);
        double lvo = 0.0;
        if (fo >= 0 && vel[a] != nullptr) {
            int r[3] = {c.i, c.j, c.k};
            r[a] += 1;
            const long long qr = at(g, r[0], r[1], r[2]);
            const double lamf = lout[qr] / gm[qr] - mu_c;
            const double vv = vel[a][fo];
            acc += ppos(vv) * lamf;
            lvo = (stp(vv) * phi[c.q] + stn(vv) * phi[qr]) * lamf;
        }
        if (lvel[a]) {
            if (assign_vel) lvel[a][c.q] = lvo;
            else if (fo >= 0 && vel[a] != nullptr) lvel[a][fo] += lvo;
        }
        // left face c-1/2: c is the right cell of the flux
        int l[3] = {c.i, c.j, c.k};
        l[a] -= 1;
        long long fl = face_idx(g, a, l[0], l[1], l[2]);
        if (fl >= 0 && vel[a] != nullptr) {
            const long long ql = at(g, l[0], l[1], l[2]);
            const double lamf = mu_c - lout[ql] / gm[ql];
            acc += pneg(vel[a][fl]) * lamf;
        }
    }
    if (assign_phi) lphi[c.q] = acc;
    else lphi[c.q] += acc;
}

// ---------------------------------------------------------------------------
// Limited velocities: from their adjoints at the cell's own and left faces,
// the antidiffusive velocities' adjoint (lut, =) at the own faces, and the
// adjoints of beta_up and beta_dn at the cell (gup, gdn)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adj_limit_cell(const Geo& g, const Cell& c, const double* __restrict__ ut,
                                               const double* __restrict__ vt, const double* __restrict__ wt,
                                               const double* __restrict__ bup, const double* __restrict__ bdn,
                                               const double (&lam_own)[3], const double (&lam_left)[3],
                                               double* __restrict__ lux, double* __restrict__ luy,
                                               double* __restrict__ luz, double& gup, double& gdn)
{
    const double* U3[3] = {ut, vt, wt};
    double* O3[3] = {lux, luy, luz};
    gup = 0.0;
    gdn = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // own face: c is its left cell
        const long long fo = face_idx(g, a, c.i, c.j, c.k);
        if (fo >= 0) {
            int r[3] = {c.i, c.j, c.k};
            r[a] += 1;
            const long long qr = at(g, r[0], r[1], r[2]);
            const double U = U3[a][fo], lam = lam_own[a];
            const double up = min2(1.0, min2(bdn[c.q], bup[qr]));
            const double dn = min2(1.0, min2(bup[c.q], bdn[qr]));
            O3[a][fo] = lam * (stp(U) * up + stn(U) * dn);
            if (U > 0.0 && first_min3(bdn[c.q], bup[qr]) == 1) gdn += lam * U;
            if (U < 0.0 && first_min3(bup[c.q], bdn[qr]) == 1) gup += lam * U;
        } else {
            // a wall's slot carries no velocity; give it a defined adjoint
            if (closed(g, a)) O3[a][c.q] = 0.0;
        }
        // left face: c is its right cell
        int l[3] = {c.i, c.j, c.k};
        l[a] -= 1;
        const long long fl = face_idx(g, a, l[0], l[1], l[2]);
        if (fl >= 0) {
            const long long ql = at(g, l[0], l[1], l[2]);
            const double U = U3[a][fl], lam = lam_left[a];
            if (U > 0.0 && first_min3(bdn[ql], bup[c.q]) == 2) gup += lam * U;
            if (U < 0.0 && first_min3(bup[ql], bdn[c.q]) == 2) gdn += lam * U;
        }
    }
}

// ---------------------------------------------------------------------------
// Bounds (max / min over the 7-point cross of psi^n and phi)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cross7(const Geo& g, int i, int j, int k, long long idx[7])
{
    idx[0] = at(g, i, j, k);
    idx[1] = at(g, i - 1, j, k);
    idx[2] = at(g, i + 1, j, k);
    idx[3] = at(g, i, j - 1, k);
    idx[4] = at(g, i, j + 1, k);
    idx[5] = at(g, i, j, k - 1);
    idx[6] = at(g, i, j, k + 1);
}

// The halo rule applied to each coordinate (each within one cell of the
// domain), without dividing a linear index back into coordinates.
struct Pt {
    int i, j, k;
    long long q;
};
__device__ __forceinline__ Pt mapped(const Geo& g, int i, int j, int k)
{
    Pt p;
    p.i = nbr(i, g.nx, g.closed_x);
    p.j = nbr(j, g.ny, g.closed_y);
    p.k = nbr(k, g.nz, g.closed_z);
    p.q = (long long)p.k * g.sz + (long long)p.j * g.sy + p.i;
    return p;
}

// Entry d (0 self, 1 -x, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z) of cell (i, j, k)'s cross.
// Branch-free: d differs from lane to lane.
__device__ __forceinline__ long long cross_entry(const Geo& g, int i, int j, int k, int d)
{
    const int di = d == 1 ? -1 : (d == 2 ? 1 : 0);
    const int dj = d == 3 ? -1 : (d == 4 ? 1 : 0);
    const int dk = d == 5 ? -1 : (d == 6 ? 1 : 0);
    return at(g, i + di, j + dj, k + dk);
}

// The bounds and, in code[2q] / code[2q+1], the first maximal / minimal
// entry e of the 14 (psi^n at the cross's 7 cells, then the iterate), the
// entry through which the adjoint of mx / mn flows.
__device__ __forceinline__ void bounds_cell(const Geo& g, const Cell& c, const double* __restrict__ psin,
                                            const double* __restrict__ phi, double& hi, double& lo, int& am, int& an)
{
    long long idx[7];
    cross7(g, c.i, c.j, c.k, idx);
    hi = psin[idx[0]];
    lo = hi;
    am = 0;
    an = 0;
    for (int e = 1; e < 14; ++e) {
        const double v = (e < 7 ? psin : phi)[idx[e % 7]];
        if (v > hi) { hi = v; am = e; }
        if (v < lo) { lo = v; an = e; }
    }
}

// (lmx, lmn) -> the cell's shares gp (of psi^n) and gf (of the iterate):
// each cell x collects from the distinct cells whose cross contains it, where
// x is the recorded first maximal / minimal entry.
__device__ __forceinline__ void adj_bounds_cell(const Geo& g, const Cell& c, const unsigned char* __restrict__ code,
                                                const double* __restrict__ lmx, const double* __restrict__ lmn,
                                                double& gp, double& gf)
{
    // Fast path: every axis periodic with >= 3 cells, or c >= 1 away from a
    // closed end.  Then the seven cells whose cross contains c are distinct,
    // and candidate y = c + step(m) reaches c only through its entry
    // opposite to m (the same candidates, order and sums as below).
    bool fast = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int n = extent(g, b), cb = b == 0 ? c.i : (b == 1 ? c.j : c.k);
        fast = fast && (closed(g, b) ? (cb >= 1 && cb <= n - 2) : n >= 3);
    }
    if (fast) {
        const long long st[3] = {1, g.sy, g.sz};
        const int cc[3] = {c.i, c.j, c.k};
        gp = gf = 0.0;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            long long yq = c.q;
            int want = 0;   // the entry of y that is c
            if (m > 0) {
                const int b = (m - 1) >> 1, s = (m & 1) ? -1 : 1;   // m = 1, 3, 5: the lower neighbour
                const int n = extent(g, b);
                int v = cc[b] + s;
                v = v < 0 ? v + n : (v >= n ? v - n : v);
                yq += (long long)(v - cc[b]) * st[b];
                want = (m & 1) ? m + 1 : m - 1;
            }
            const int am = code[2 * yq], an = code[2 * yq + 1];
            if (am % 7 == want) (am < 7 ? gp : gf) += lmx[yq];
            if (an % 7 == want) (an < 7 ? gp : gf) += lmn[yq];
        }
        return;
    }
    // the cells whose cross contains c (the cross is symmetric)
    const Pt cand[7] = {mapped(g, c.i, c.j, c.k),     mapped(g, c.i - 1, c.j, c.k), mapped(g, c.i + 1, c.j, c.k),
                        mapped(g, c.i, c.j - 1, c.k), mapped(g, c.i, c.j + 1, c.k), mapped(g, c.i, c.j, c.k - 1),
                        mapped(g, c.i, c.j, c.k + 1)};
    gp = gf = 0.0;
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        bool dup = false;
#pragma unroll
        for (int m2 = 0; m2 < m; ++m2) dup = dup || cand[m2].q == cand[m].q;
        if (dup) continue;
        const Pt& y = cand[m];
        const int am = code[2 * y.q], an = code[2 * y.q + 1];
        if (cross_entry(g, y.i, y.j, y.k, am % 7) == c.q) (am < 7 ? gp : gf) += lmx[y.q];
        if (cross_entry(g, y.i, y.j, y.k, an % 7) == c.q) (an < 7 ? gp : gf) += lmn[y.q];
    }
}

// ---------------------------------------------------------------------------
// Limiter coefficients beta_up = (mx - phi) G / (in + eps),
// beta_dn = (phi - mn) G / (out + eps).
// Per cell (adj_beta1_cell): the adjoints of in and out (lin, lout), of mx
// and mn, and beta's direct dependence on phi.  Gathered (adj_inout_cell):
// in and out's dependence on phi and on the antidiffusive velocities.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void in_out(const Geo& g, const Cell& c, const double* __restrict__ phi,
                                       const double* const U3[3], double& in, double& out)
{
    double fin[3], fout[3];
    const double pc = phi[c.q];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int l[3] = {c.i, c.j, c.k}, r[3] = {c.i, c.j, c.k};
        l[a] -= 1;
        r[a] += 1;
        const long long fr = face_idx(g, a, c.i, c.j, c.k);
        const long long fl = face_idx(g, a, l[0], l[1], l[2]);
        const double vr = fr < 0 ? 0.0 : U3[a][fr];
        const double vl = fl < 0 ? 0.0 : U3[a][fl];
        fin[a] = ppos(vl) * phi[at(g, l[0], l[1], l[2])] - pneg(vr) * phi[at(g, r[0], r[1], r[2])];
        fout[a] = ppos(vr) * pc - pneg(vl) * pc;
    }
    in = (fin[0] + fin[1]) + fin[2];
    out = (fout[0] + fout[1]) + fout[2];
}

__device__ __forceinline__ void adj_beta1_cell(const Geo& g, const Cell& c, double eps, const double* __restrict__ phi,
                                               const double* __restrict__ ut, const double* __restrict__ vt,
                                               const double* __restrict__ wt, double mx, double mn,
                                               const double* __restrict__ gm, double gu, double gd,
                                               double* __restrict__ lin,
                                               double* __restrict__ lout, double* __restrict__ lmx,
                                               double* __restrict__ lmn, double* __restrict__ lphi)
{
    const double* U3[3] = {ut, vt, wt};
    double in, out;
    in_out(g, c, phi, U3, in, out);
    const double rin = rcp_nr(in + eps), rout = rcp_nr(out + eps);
    const double G = gm[c.q], pc = phi[c.q];
    const double bu = ((mx - pc) * G) * rin;
    const double bd = ((pc - mn) * G) * rout;
    lmx[c.q] = gu * G * rin;
    lmn[c.q] = -(gd * G * rout);
    lphi[c.q] += -gu * G * rin + gd * G * rout;
    lin[c.q] = -gu * bu * rin;
    lout[c.q] = -gd * bd * rout;
}

// in(c)  = sum_a [U(c-1/2)]+ phi(c-1) - [U(c+1/2)]- phi(c+1)
// out(c) = sum_a ([U(c+1/2)]+ - [U(c-1/2)]-) phi(c)
__device__ __forceinline__ double adj_inout_cell(const Geo& g, const Cell& c, const double* __restrict__ phi,
                                                 const double* __restrict__ ut, const double* __restrict__ vt,
                                                 const double* __restrict__ wt, const double* __restrict__ lin,
                                                 const double* __restrict__ lout, double (&dl)[3])
{
    const double* U3[3] = {ut, vt, wt};
    const double pc = phi[c.q];
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dl[a] = 0.0;
        int l[3] = {c.i, c.j, c.k}, r[3] = {c.i, c.j, c.k};
        l[a] -= 1;
        r[a] += 1;
        const long long fo = face_idx(g, a, c.i, c.j, c.k);
        const long long fl = face_idx(g, a, l[0], l[1], l[2]);
        if (fo >= 0) {
            const long long qr = at(g, r[0], r[1], r[2]);
            const double U = U3[a][fo];
            // c is the left cell of its own face: inflow term of r, outflow term of c
            acc += lin[qr] * ppos(U) + lout[c.q] * ppos(U);
            // the face's own adjoint: in(r), in(c), out(c), out(r)
            dl[a] = lin[qr] * stp(U) * pc - lin[c.q] * stn(U) * phi[qr] + lout[c.q] * stp(U) * pc -
                    lout[qr] * stn(U) * phi[qr];
        }
        if (fl >= 0) {
            const long long ql = at(g, l[0], l[1], l[2]);
            const double U = U3[a][fl];
            // c is the right cell of its left face: inflow term of l, outflow term of c
            acc += -lin[ql] * pneg(U) - lout[c.q] * pneg(U);
        }
    }
    return acc;
}

// The limiter's adjoint in two gathers.  First, per cell, fused with the
// pass's donor-cell adjoint: dJ/dphi's donor-cell terms (lphi, =) and the
// adjoints of the limited velocities at the cell's own and left faces, formed
// in registers: their donor-cell part from lnext, phi and G (at the left face
// the same expression, operand for operand, that the left cell forms for its
// own face, so both agree bitwise) plus, unless assign_vel, what the next
// pass's antidiffusive-velocity adjoint left in lvx/lvy/lvz.  From them the
// antidiffusive velocities' adjoint (lut, =) and, from the adjoints of beta
// it yields (kept in registers), those of in, out, mx and mn (=) and beta's
// direct dependence on the iterate (lphi, +=).
__global__ void __launch_bounds__(256) k_adj_donor_limit_beta(
    Geo g, double eps, const double* __restrict__ phi, const double* __restrict__ vlx, const double* __restrict__ vly,
    const double* __restrict__ vlz, const double* __restrict__ gm, const double* __restrict__ lnext,
    const double* __restrict__ lvx, const double* __restrict__ lvy, const double* __restrict__ lvz, int assign_vel,
    const double* __restrict__ ut, const double* __restrict__ vt, const double* __restrict__ wt,
    const double* __restrict__ bup, const double* __restrict__ bdn, const double* __restrict__ psin,
    unsigned char* __restrict__ code, double* __restrict__ lux, double* __restrict__ luy, double* __restrict__ luz,
    double* __restrict__ lin, double* __restrict__ lout, double* __restrict__ lmx, double* __restrict__ lmn,
    double* __restrict__ lphi)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    const double* vel[3] = {vlx, vly, vlz};
    const double* L3[3] = {lvx, lvy, lvz};
    double acc = lnext[c.q];
    const double mu_c = lnext[c.q] / gm[c.q];
    double lam_own[3], lam_left[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // own face c+1/2: the flux leaves c and enters r
        lam_own[a] = 0.0;
        const long long fo = face_idx(g, a, c.i, c.j, c.k);
        if (fo >= 0) {
            int r[3] = {c.i, c.j, c.k};
            r[a] += 1;
            const long long qr = at(g, r[0], r[1], r[2]);
            const double lamf = lnext[qr] / gm[qr] - mu_c;
            const double vv = vel[a][fo];
            acc += ppos(vv) * lamf;
            lam_own[a] = (stp(vv) * phi[c.q] + stn(vv) * phi[qr]) * lamf;
            if (!assign_vel) lam_own[a] += L3[a][fo];
        }
        // left face c-1/2: c is the right cell of the flux; its donor part
        // is the same expression the left cell forms for its own face
        lam_left[a] = 0.0;
        int l[3] = {c.i, c.j, c.k};
        l[a] -= 1;
        const long long fl = face_idx(g, a, l[0], l[1], l[2]);
        if (fl >= 0) {
            const long long ql = at(g, l[0], l[1], l[2]);
            const double lamf = mu_c - lnext[ql] / gm[ql];
            const double vv = vel[a][fl];
            acc += pneg(vv) * lamf;
            lam_left[a] = (stp(vv) * phi[ql] + stn(vv) * phi[c.q]) * lamf;
            if (!assign_vel) lam_left[a] += L3[a][fl];
        }
    }
    lphi[c.q] = acc;
    double gup, gdn;
    adj_limit_cell(g, c, ut, vt, wt, bup, bdn, lam_own, lam_left, lux, luy, luz, gup, gdn);
    // the bounds of the cell and the first extremal entries they came from
    // (code: read by the bounds' gather in k_adj_inout_bounds_antidiff1)
    double hi, lo;
    int am, an;
    bounds_cell(g, c, psin, phi, hi, lo, am, an);
    code[2 * c.q] = (unsigned char)am;
    code[2 * c.q + 1] = (unsigned char)an;
    adj_beta1_cell(g, c, eps, phi, ut, vt, wt, hi, lo, gm, gup, gdn, lin, lout, lmx, lmn, lphi);
}

// Second, gathering from the neighbours: in and out's dependence on the
// iterate and on the antidiffusive velocities (lphi +=, lut +=), and the
// bounds' routing to psi^n (lpsin: = for its first contribution in a step,
// else +=) and to the iterate (lphi +=).

// ---------------------------------------------------------------------------
// Antidiffusive velocity
//   U~ = (|U| - U^2/Gf) A - (U/Gf) (Vb_1 B_1 + Vb_2 B_2)
//   A = (pR - pL)/(pR + pL + eps), B_t = (Sp - Sm)/(2 (Sp + Sm + eps)),
//   Sp = phi(R+t) + phi(L+t), Sm = phi(R-t) + phi(L-t),
//   Vb_t = (V_t(L) + V_t(R) + V_t(L-t) + V_t(R-t))/4, Gf = (G(L) + G(R))/2.
// Kernel 1 stores, per face (axis a, left cell y), lambda times:
//   s0 dU~/dpR, s1/s2 dU~/dSp_1, dU~/dSm_1, s3/s4 the same for the second
//   transverse axis, s5/s6 dU~/dV_t of each of the four faces of transverse
//   axis t.  The two terms that belong to the face's own cell and face go
//   straight into the adjoints instead: lambda dU~/dpL is added to dJ/dphi
//   at y, and lambda dU~/dU to the velocity adjoint (assigned when
//   assign_vel, else added; a closed wall's unused slot gets 0 when
//   assigned).  Kernel 2 then adds the gathered terms to both.
// ---------------------------------------------------------------------------
constexpr int kSlots = 7;

// Kernel 1's work at the face c + 1/2 along axis a, given the adjoint lam of
// its antidiffusive velocity: the seven slot values (s), lambda dU~/dU (ldu)
// and lambda dU~/dpL (returned).  False (and nothing set) at a closed wall.
__device__ __forceinline__ bool antidiff1_face(const Geo& g, const Cell& c, int a, double eps,
                                               const double* __restrict__ phi, const double* const (&vel)[3],
                                               const double* __restrict__ gm, double lam, double (&s)[kSlots],
                                               double& ldu, double& own)
{
    const long long fo = face_idx(g, a, c.i, c.j, c.k);   // c.q when valid
    if (fo < 0) return false;
    int R[3] = {c.i, c.j, c.k};
    R[a] += 1;
    const double pL = phi[c.q], pR = phi[at(g, R[0], R[1], R[2])];
    const double D0 = (pR + pL) + eps;
    const double rD0 = rcp_nr(D0);
    const double A = (pR - pL) * rD0;
    double B[2], Vb[2], rDt[2], Sp[2], Sm[2];
    int sidx = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (t == a) continue;
        int Lp[3] = {c.i, c.j, c.k}, Rp[3] = {R[0], R[1], R[2]};
        int Lm[3] = {c.i, c.j, c.k}, Rm[3] = {R[0], R[1], R[2]};
        Lp[t] += 1; Rp[t] += 1; Lm[t] -= 1; Rm[t] -= 1;
        Sp[sidx] = phi[at(g, Rp[0], Rp[1], Rp[2])] + phi[at(g, Lp[0], Lp[1], Lp[2])];
        Sm[sidx] = phi[at(g, Rm[0], Rm[1], Rm[2])] + phi[at(g, Lm[0], Lm[1], Lm[2])];
        rDt[sidx] = rcp_nr((Sp[sidx] + Sm[sidx]) + eps);
        B[sidx] = 0.5 * ((Sp[sidx] - Sm[sidx]) * rDt[sidx]);
        const long long f0 = face_idx(g, t, c.i, c.j, c.k), f1 = face_idx(g, t, R[0], R[1], R[2]);
        const long long f2 = face_idx(g, t, Lm[0], Lm[1], Lm[2]), f3 = face_idx(g, t, Rm[0], Rm[1], Rm[2]);
        const double* vt = vel[t];
        const double v0 = (f0 < 0 || !vt) ? 0.0 : vt[f0], v1 = (f1 < 0 || !vt) ? 0.0 : vt[f1];
        const double v2 = (f2 < 0 || !vt) ? 0.0 : vt[f2], v3 = (f3 < 0 || !vt) ? 0.0 : vt[f3];
        Vb[sidx] = 0.25 * ((v0 + v1) + (v2 + v3));
        ++sidx;
    }
    const double rGf = rcp_nr(0.5 * (gm[c.q] + gm[at(g, R[0], R[1], R[2])]));
    const double U = vel[a] ? vel[a][fo] : 0.0;
    const double S = (Vb[0] * B[0]) + (Vb[1] * B[1]);
    const double dU = (sgn(U) - 2.0 * U * rGf) * A - S * rGf;
    const double dA = (U < 0.0 ? -U : U) - (U * U) * rGf;
    const double dS = -U * rGf;
    const double gA = lam * dA;
    const double r2 = rD0 * rD0;
    s[0] = gA * (2.0 * pL + eps) * r2;
    own = -(gA * (2.0 * pR + eps) * r2);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double gB = lam * dS * Vb[q];
        const double rt2 = rDt[q] * rDt[q];
        s[1 + 2 * q] = gB * (0.5 * (2.0 * Sm[q] + eps) * rt2);
        s[2 + 2 * q] = gB * (-0.5 * (2.0 * Sp[q] + eps) * rt2);
        s[5 + q] = 0.25 * (lam * dS * B[q]);
    }
    ldu = lam * dU;
    return true;
}

// Kernel 1's work at one cell, given the adjoints lam of the antidiffusive
// velocities at its three own faces; returns lambda dU~/dpL summed over them.
__device__ __forceinline__ double antidiff1_cell(const Geo& g, const Cell& c, double eps, const double* __restrict__ phi,
                                                 const double* __restrict__ u, const double* __restrict__ v,
                                                 const double* __restrict__ w, const double* __restrict__ gm,
                                                 const double (&lam_face)[3], double* __restrict__ slots,
                                                 long long field, double* __restrict__ lu, double* __restrict__ lv,
                                                 double* __restrict__ lw, bool assign_vel)
{
    const double* const vel[3] = {u, v, w};
    double* lvel[3] = {lu, lv, lw};
    double own = 0.0;   // lambda dU~/dpL of the cell's three faces
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double* sp = slots + (long long)a * kSlots * field + c.q;
        double s[kSlots], ldu, own_a;
        if (!antidiff1_face(g, c, a, eps, phi, vel, gm, lam_face[a], s, ldu, own_a)) {
            for (int e = 0; e < kSlots; ++e) sp[e * field] = 0.0;
            if (lvel[a] && assign_vel) lvel[a][c.q] = 0.0;   // a closed wall's unused slot
            continue;
        }
        own += own_a;
#pragma unroll
        for (int e = 0; e < kSlots; ++e) sp[e * field] = s[e];
        if (lvel[a]) {
            if (assign_vel) lvel[a][c.q] = ldu;
            else lvel[a][c.q] += ldu;
        }
    }
    return own;
}

__global__ void __launch_bounds__(256) k_adj_antidiff1(Geo g, double eps, const double* __restrict__ phi,
                                                       const double* __restrict__ u, const double* __restrict__ v,
                                                       const double* __restrict__ w, const double* __restrict__ gm,
                                                       const double* __restrict__ lux, const double* __restrict__ luy,
                                                       const double* __restrict__ luz, double* __restrict__ slots,
                                                       long long field, double* __restrict__ lphi,
                                                       double* __restrict__ lu, double* __restrict__ lv,
                                                       double* __restrict__ lw, bool assign_vel)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    const double lam[3] = {lux[c.q], luy[c.q], luz[c.q]};
    lphi[c.q] += antidiff1_cell(g, c, eps, phi, u, v, w, gm, lam, slots, field, lu, lv, lw, assign_vel);
}

// A limited pass: the limiter's second gather (in / out and the bounds)
// fused with kernel 1.  The antidiffusive velocities' adjoint at the cell's
// own faces is what the limiter's first kernel left in lutx/luty/lutz plus
// the in / out terms formed here, kept in registers for kernel 1's work (the
// same sums, in the same order, as adding it to lut and reading it back).
// The bounds route to psi^n (lpsin: = when assign_psin, else +=); dJ/dphi
// gains the in / out and bound terms and then kernel 1's own-cell term.
__global__ void __launch_bounds__(256) k_adj_inout_bounds_antidiff1(
    Geo g, double eps, const double* __restrict__ phi, const double* __restrict__ ut, const double* __restrict__ vt,
    const double* __restrict__ wt, const double* __restrict__ lin, const double* __restrict__ lout,
    const unsigned char* __restrict__ code, const double* __restrict__ lmx, const double* __restrict__ lmn,
    const double* __restrict__ lutx, const double* __restrict__ luty, const double* __restrict__ lutz,
    double* __restrict__ lpsin, int assign_psin, const double* __restrict__ pu, const double* __restrict__ pv,
    const double* __restrict__ pw, const double* __restrict__ gm, double* __restrict__ slots, long long field,
    double* __restrict__ lphi, double* __restrict__ lu, double* __restrict__ lv, double* __restrict__ lw,
    bool assign_vel)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    double dl[3];
    const double acc = adj_inout_cell(g, c, phi, ut, vt, wt, lin, lout, dl);
    double gp, gf;
    adj_bounds_cell(g, c, code, lmx, lmn, gp, gf);
    if (assign_psin) lpsin[c.q] = gp;
    else lpsin[c.q] += gp;
    const double lam[3] = {lutx[c.q] + dl[0], luty[c.q] + dl[1], lutz[c.q] + dl[2]};
    const double own = antidiff1_cell(g, c, eps, phi, pu, pv, pw, gm, lam, slots, field, lu, lv, lw, assign_vel);
    lphi[c.q] = (lphi[c.q] + (acc + gf)) + own;
}

// Kernel 2: each cell x gathers the slots of the faces that read phi(x), and
// of the faces that read the velocities of its three own faces.  Candidate
// faces come from the stencil offsets; every candidate's actual inputs are
// recomputed through the halo rules and compared with x, so wrap, clamp and
// tiny grids (where one cell fills several input positions) are exact.
// dJ/dphi at cell x from the faces along axis A (the general path of
// k_adj_antidiff2): the distinct faces y whose 10 stencil positions (L, R,
// L+-t1, R+-t1, L+-t2, R+-t2 after the halo rule) include x, each position
// that is x adding that position's partial derivative.  Position L is the
// cell y itself, so it is x only for the face y = x, whose term kernel 1
// has added already.
template <int A>
__device__ __forceinline__ double adj_antidiff_general_axis(const Geo& g, const int (&Yt)[3][3],
                                                            const int (&Tt)[3][3][3], const Cell& c,
                                                            const double* __restrict__ slots, long long field)
{
    constexpr int t1 = A == 0 ? 1 : 0, t2 = A == 2 ? 1 : 2;
    // stencil offsets of face (A, y) relative to its left cell, and their slots
    int off[10][3], slot_of[10];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        off[e][0] = off[e][1] = off[e][2] = 0;
        off[e][A] = e;
        slot_of[e] = 0;   // R (L, e = 0, is never looked up)
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int n = 2 + 4 * q + 2 * h + e;
                off[n][0] = off[n][1] = off[n][2] = 0;
                off[n][A] = e;
                off[n][q == 0 ? t1 : t2] = h == 0 ? 1 : -1;
                slot_of[n] = 1 + 2 * q + h;
            }
    const int xc[3] = {c.i, c.j, c.k};
    const int nA = extent(g, A), clA = closed(g, A);
    const double* sA = slots + (long long)A * kSlots * field;
    double acc = 0.0;
    long long seen[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) {
        // candidate face y = x - off[m] (mapped)
        const int yi = Yt[0][off[m][0] + 1], yj = Yt[1][off[m][1] + 1], yk = Yt[2][off[m][2] + 1];
        const long long y = (long long)yk * g.sz + (long long)yj * g.sy + yi;
        seen[m] = y;
        bool dup = false;
#pragma unroll
        for (int s2 = 0; s2 < m; ++s2) dup = dup || seen[s2] == y;
        const int ya = A == 0 ? yi : (A == 1 ? yj : yk);
        if (dup || (clA && ya >= nA - 1)) continue;     // counted already / wall: U~ is the constant 0
#pragma unroll
        for (int e = 1; e < 10; ++e) {
            const bool hit = Tt[0][off[m][0] + 1][off[e][0] + 1] == xc[0] &&
                             Tt[1][off[m][1] + 1][off[e][1] + 1] == xc[1] &&
                             Tt[2][off[m][2] + 1][off[e][2] + 1] == xc[2];
            if (hit) acc += sA[slot_of[e] * field + y];
        }
    }
    return acc;
}

// 6 waves per SIMD: 80 VGPRs with no spills (unbounded it takes 82, 5 waves)
// general_only: only the cells of the general path (the k-marching kernel
// of adjoint_march.hpp has gathered the others).
__global__ void __launch_bounds__(256, 6) k_adj_antidiff2(Geo g, const double* __restrict__ slots, long long field,
                                                       double* __restrict__ lphi, double* __restrict__ lu,
                                                       double* __restrict__ lv, double* __restrict__ lw,
                                                       int general_only)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    double* lvel[3] = {lu, lv, lw};
    const long long x = c.q;

    // Fast path: no wrap or clamp collision anywhere in the stencil (every
    // axis periodic with >= 4 cells, or the cell >= 2 away from a closed
    // end).  Then each candidate face reads x exactly at the position that
    // names it, and each transverse velocity read hits x's face once.
    bool fast = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int n = extent(g, b), cb = b == 0 ? c.i : (b == 1 ? c.j : c.k);
        fast = fast && (closed(g, b) ? (cb >= 2 && cb <= n - 3) : n >= 4);
    }
    if (fast) {
        if (general_only) return;
        const long long st[3] = {1, g.sy, g.sz};
        const int cc[3] = {c.i, c.j, c.k};
        // offset of x - o along axis b (periodic wrap; closed axes are interior here)
        auto shifted = [&](int b, int o) -> long long {
            const int n = extent(g, b);
            int v = cc[b] - o;
            if (v < 0) v += n;
            else if (v >= n) v -= n;
            return (long long)(v - cc[b]) * st[b];
        };
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const double* s = slots + (long long)a * kSlots * field;
            const long long da = shifted(a, 1);
            // R = x (face at x - a); L = x was added by kernel 1
            acc += s[0 * field + x + da];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int t = q == 0 ? t1 : t2;
                const long long dp = shifted(t, 1), dm = shifted(t, -1);
                // x = L + t or R + t: faces at x - t and x - t - a (slot Sp)
                acc += s[(1 + 2 * q) * field + x + dp] + s[(1 + 2 * q) * field + x + dp + da];
                // x = L - t or R - t: faces at x + t and x + t - a (slot Sm)
                acc += s[(2 + 2 * q) * field + x + dm] + s[(2 + 2 * q) * field + x + dm + da];
            }
        }
        lphi[x] += acc;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (!lvel[t]) continue;
            double accv = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (a == t) continue;
                const int q = (t == (a == 0 ? 1 : 0)) ? 0 : 1;
                const double* s6 = slots + ((long long)a * kSlots + 5 + q) * field;
                const long long da = shifted(a, 1), dt = shifted(t, -1);
                // face (t, x) is read by faces (a, y) at y = x, x - a, x + t, x - a + t
                accv += (s6[x] + s6[x + da]) + (s6[x + dt] + s6[x + da + dt]);
            }
            lvel[t][x] += accv;
        }
        return;
    }

    // General path (a closed end within two cells on some axis).  The halo
    // rule maps each coordinate independently, so the candidate faces and
    // their stencil positions are looked up in per-axis tables of mapped
    // coordinates: Y[b][o] = nbr(x_b - o) and T[b][o1][o2] = nbr(Y[b][o1] + o2)
    // for offsets o, o1, o2 in {-1, 0, 1}.
    int Yt[3][3], Tt[3][3][3];
    {
        const int xc[3] = {c.i, c.j, c.k};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int n = extent(g, b), cl = closed(g, b);
#pragma unroll
            for (int o1 = 0; o1 < 3; ++o1) {
                Yt[b][o1] = nbr(xc[b] - (o1 - 1), n, cl);
#pragma unroll
                for (int o2 = 0; o2 < 3; ++o2) Tt[b][o1][o2] = nbr(Yt[b][o1] + (o2 - 1), n, cl);
            }
        }
    }
    double acc = adj_antidiff_general_axis<0>(g, Yt, Tt, c, slots, field) +
                 adj_antidiff_general_axis<1>(g, Yt, Tt, c, slots, field);
    acc += adj_antidiff_general_axis<2>(g, Yt, Tt, c, slots, field);
    lphi[x] += acc;

    // velocities of x's own faces: face (t, x) is read as the own velocity of
    // face (t, x) and in the transverse averages of faces (a != t, y) at
    // V_t(y), V_t(y+a), V_t(y-t), V_t(y+a-t)
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (!lvel[t]) continue;
        const long long fx = face_idx(g, t, c.i, c.j, c.k);
        if (fx < 0) continue;   // a closed wall's unused slot (kernel 1 wrote it)
        double accv = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == t) continue;
            // position of t among a's transverse axes in increasing order
            const int q = (t == (a == 0 ? 1 : 0)) ? 0 : 1;
            int o4[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            o4[1][a] = 1;
            o4[2][t] = -1;
            o4[3][a] = 1;
            o4[3][t] = -1;
            long long seen[4] = {-1, -1, -1, -1};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                int yc[3] = {c.i - o4[m][0], c.j - o4[m][1], c.k - o4[m][2]};
                // the face coordinate along t stays a face index: map the
                // other axes only (wrap / clamp), then require a valid cell
                int yt = yc[t];
                const int nt = extent(g, t);
                if (yt < 0) {
                    if (closed(g, t)) continue;
                    yt += nt;
                } else if (yt >= nt) {
                    if (closed(g, t)) continue;
                    yt -= nt;
                }
                yc[t] = yt;
                const Pt yp = mapped(g, yc[0], yc[1], yc[2]);
                const long long y = yp.q;
                seen[m] = y;
                bool dup = false;
#pragma unroll
                for (int s2 = 0; s2 < m; ++s2) dup = dup || seen[s2] == y;
                if (dup) continue;
                const int yk = yp.k, yj = yp.j, yi = yp.i;
                if (face_idx(g, a, yi, yj, yk) < 0) continue;
                int ry[3] = {yi, yj, yk};
                ry[a] += 1;
                int lm[3] = {yi, yj, yk};
                lm[t] -= 1;
                int rm[3] = {ry[0], ry[1], ry[2]};
                rm[t] -= 1;
                int hits = (face_idx(g, t, yi, yj, yk) == fx) + (face_idx(g, t, ry[0], ry[1], ry[2]) == fx) +
                           (face_idx(g, t, lm[0], lm[1], lm[2]) == fx) + (face_idx(g, t, rm[0], rm[1], rm[2]) == fx);
                if (hits) accv += hits * slots[((long long)a * kSlots + 5 + q) * field + y];
            }
        }
        lvel[t][fx] += accv;
    }
}

#pragma clang fp contract(on)

}  // namespace adj
}  // namespace mpdata
