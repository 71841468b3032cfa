// stages.hpp -- one kernel per stage of an MPDATA pass, one thread per cell.
//
// The straightforward form of the step: every stage reads its inputs from
// HBM and writes its outputs back.  It is built without FMA contraction and
// evaluates every expression in the scheme's order, so its FP64 results are
// the scheme's rounded results exactly; it serves any iteration count and
// boundary combination.  The fused k-marching kernels (fused.hpp) are the
// fast path for the common configurations.
//
// Stages (per pass): donor-cell flux, divergence and update (paper,
// Section 5, Listings 4-8); antidiffusive pseudo-velocities; limiter bounds
// and coefficients; limited velocities (the MPDATA iterations and the
// non-oscillatory option the paper leaves to its companion deliverable).
#pragma once

#include "common.hpp"

namespace mpdata {
namespace stages {

#pragma clang fp contract(off)

struct Cell {
    int i, j, k;
    long long q;
};

__device__ __forceinline__ bool cell_of_thread(const Geo& g, Cell& c)
{
    c.i = blockIdx.x * blockDim.x + threadIdx.x;
    c.j = blockIdx.y * blockDim.y + threadIdx.y;
    c.k = blockIdx.z;
    if (c.i >= g.nx || c.j >= g.ny) return false;
    c.q = (long long)c.k * g.sz + (long long)c.j * g.sy + c.i;
    return true;
}

// Linear index of (i, j, k) after the halo rule on each axis (inputs within
// one cell of the domain).
__device__ __forceinline__ long long at(const Geo& g, int i, int j, int k)
{
    return (long long)nbr(k, g.nz, g.closed_z) * g.sz + (long long)nbr(j, g.ny, g.closed_y) * g.sy +
           nbr(i, g.nx, g.closed_x);
}

// Face value along `axis` of the face c_axis + 1/2 at column (i, j, k); the
// coordinates across the axis go through the halo rule, the one along it may
// be -1 .. n-1.
template <class T>
__device__ __forceinline__ T face(const Geo& g, const T* __restrict__ a, int axis, int i, int j, int k)
{
    if (axis == 0) {
        long long base = (long long)nbr(k, g.nz, g.closed_z) * g.sz + (long long)nbr(j, g.ny, g.closed_y) * g.sy;
        return face_at(a, base, 1, i, g.nx, g.closed_x);
    }
    if (axis == 1) {
        long long base = (long long)nbr(k, g.nz, g.closed_z) * g.sz + nbr(i, g.nx, g.closed_x);
        return face_at(a, base, g.sy, j, g.ny, g.closed_y);
    }
    long long base = (long long)nbr(j, g.ny, g.closed_y) * g.sy + nbr(i, g.nx, g.closed_x);
    return face_at(a, base, g.sz, k, g.nz, g.closed_z);
}

__device__ __forceinline__ int extent(const Geo& g, int axis) { return axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz; }
__device__ __forceinline__ int closed(const Geo& g, int axis)
{
    return axis == 0 ? g.closed_x : axis == 1 ? g.closed_y : g.closed_z;
}

// Donor-cell update of one cell: phi - div(F)/G with F = [u]+ phi_left + [u]- phi_right.
template <class T>
__device__ __forceinline__ T donor_cell(const Geo& g, const Cell& c, const T* __restrict__ phi,
                                        const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
                                        const T* __restrict__ gm)
{
    const T* vel[3] = {u, v, w};
    const T pc = phi[c.q];
    T dif[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (vel[a] == nullptr) {   // an absent velocity field is all zero
            dif[a] = T(0) - T(0);
            continue;
        }
        int r[3] = {c.i, c.j, c.k}, l[3] = {c.i, c.j, c.k};
        r[a] += 1;
        l[a] -= 1;
        T ur = face(g, vel[a], a, c.i, c.j, c.k);
        T ul = face(g, vel[a], a, l[0], l[1], l[2]);
        T pr = phi[at(g, r[0], r[1], r[2])];
        T pl = phi[at(g, l[0], l[1], l[2])];
        T fr = (pos_part(ur) * pc) + (neg_part(ur) * pr);
        T fl = (pos_part(ul) * pl) + (neg_part(ul) * pc);
        dif[a] = fr - fl;
    }
    return pc - ((dif[0] + dif[1]) + dif[2]) / gm[c.q];
}

// Donor-cell pass over one problem.
template <class T>
__global__ void __launch_bounds__(256) k_donor(Geo g, const T* __restrict__ phi, const T* __restrict__ u,
                                               const T* __restrict__ v, const T* __restrict__ w,
                                               const T* __restrict__ gm, T* __restrict__ out)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    out[c.q] = donor_cell(g, c, phi, u, v, w, gm);
}

// One (problem, tracer set) of a batched copy: entry e owns the global cells
// [begin, begin + tracers * cells).
template <class T>
struct DonorEntry {
    Geo geo;
    const T* phi;      // tracer 0 (tracer t at + t * stride)
    T* out;
    const T* u;
    const T* v;
    const T* w;        // may be NULL
    const T* g;
    long long begin, cells, stride;
    int tracers;
};

// Antidiffusive pseudo-velocities at the three own faces of every cell.
template <class T>
__global__ void __launch_bounds__(256) k_antidiff(Geo g, T eps, const T* __restrict__ phi,
                                                  const T* __restrict__ u, const T* __restrict__ v,
                                                  const T* __restrict__ w, const T* __restrict__ gm,
                                                  T* __restrict__ ut, T* __restrict__ vt, T* __restrict__ wt)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    const T* vel[3] = {u, v, w};
    T* outv[3] = {ut, vt, wt};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int L[3] = {c.i, c.j, c.k};
        if (closed(g, a) && L[a] == extent(g, a) - 1) {
            outv[a][c.q] = T(0);
            continue;
        }
        int R[3] = {c.i, c.j, c.k};
        R[a] += 1;
        const T pL = phi[c.q];
        const T pR = phi[at(g, R[0], R[1], R[2])];
        const T A = (pR - pL) / ((pR + pL) + eps);
        T B[2], Vb[2];
        int s = 0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t == a) continue;
            int Lp[3] = {L[0], L[1], L[2]}, Rp[3] = {R[0], R[1], R[2]};
            int Lm[3] = {L[0], L[1], L[2]}, Rm[3] = {R[0], R[1], R[2]};
            Lp[t] += 1;
            Rp[t] += 1;
            Lm[t] -= 1;
            Rm[t] -= 1;
            const T Sp = phi[at(g, Rp[0], Rp[1], Rp[2])] + phi[at(g, Lp[0], Lp[1], Lp[2])];
            const T Sm = phi[at(g, Rm[0], Rm[1], Rm[2])] + phi[at(g, Lm[0], Lm[1], Lm[2])];
            B[s] = T(0.5) * ((Sp - Sm) / ((Sp + Sm) + eps));
            // R may sit across a periodic wrap along a; map it before reading faces
            int Rw[3] = {R[0], R[1], R[2]};
            Rw[a] = nbr(R[a], extent(g, a), closed(g, a));
            int Rwm[3] = {Rw[0], Rw[1], Rw[2]};
            Rwm[t] -= 1;
            Vb[s] = T(0.25) * ((face(g, vel[t], t, L[0], L[1], L[2]) + face(g, vel[t], t, Rw[0], Rw[1], Rw[2])) +
                               (face(g, vel[t], t, Lm[0], Lm[1], Lm[2]) + face(g, vel[t], t, Rwm[0], Rwm[1], Rwm[2])));
            ++s;
        }
        const T Gf = T(0.5) * (gm[c.q] + gm[at(g, R[0], R[1], R[2])]);
        const T U = vel[a][c.q];
        const T au = U < T(0) ? -U : U;
        outv[a][c.q] = ((au - (U * U) / Gf) * A) - ((U / Gf) * ((Vb[0] * B[0]) + (Vb[1] * B[1])));
    }
}

// Limiter: 7-point bounds of psi^n and phi, in/out antidiffusive fluxes and
// the coefficients beta_up = (max - phi) G / (in + eps),
// beta_dn = (phi - min) G / (out + eps).  The ratio is taken in FP64 for
// both storage types.
template <class T>
__global__ void __launch_bounds__(256) k_beta(Geo g, double eps, const T* __restrict__ psin,
                                              const T* __restrict__ phi, const T* __restrict__ ut,
                                              const T* __restrict__ vt, const T* __restrict__ wt,
                                              const T* __restrict__ gm, T* __restrict__ bup, T* __restrict__ bdn)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    const T* vel[3] = {ut, vt, wt};
    const T pc = phi[c.q];
    T hi = psin[c.q], lo = hi;
    hi = max2(hi, pc);
    lo = min2(lo, pc);
    T fin[3], fout[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int r[3] = {c.i, c.j, c.k}, l[3] = {c.i, c.j, c.k};
        r[a] += 1;
        l[a] -= 1;
        long long qr = at(g, r[0], r[1], r[2]), ql = at(g, l[0], l[1], l[2]);
        const T pr = phi[qr], pl = phi[ql];
        hi = max2(hi, max2(max2(psin[qr], psin[ql]), max2(pr, pl)));
        lo = min2(lo, min2(min2(psin[qr], psin[ql]), min2(pr, pl)));
        const T vr = face(g, vel[a], a, c.i, c.j, c.k);
        const T vl = face(g, vel[a], a, l[0], l[1], l[2]);
        const T fp_l = pos_part(vl) * pl;
        const T fm_l = neg_part(vl) * pc;
        const T fp_r = pos_part(vr) * pc;
        const T fm_r = neg_part(vr) * pr;
        fin[a] = fp_l - fm_r;
        fout[a] = fp_r - fm_l;
    }
    const double in = (double)((fin[0] + fin[1]) + fin[2]);
    const double out = (double)((fout[0] + fout[1]) + fout[2]);
    const T gc = gm[c.q];
    bup[c.q] = (T)((double)((hi - pc) * gc) / (in + eps));
    bdn[c.q] = (T)((double)((pc - lo) * gc) / (out + eps));
}

// Limited velocities from the antidiffusive ones (ul, vl, wl may be ut, vt,
// wt themselves: each thread reads and writes only its own three faces).
template <class T>
__global__ void __launch_bounds__(256) k_limit(Geo g, const T* ut, const T* vt, const T* wt, T* ul, T* vl, T* wl,
                                               const T* __restrict__ bup, const T* __restrict__ bdn)
{
    Cell c;
    if (!cell_of_thread(g, c)) return;
    const T* vel[3] = {ut, vt, wt};
    T* lim[3] = {ul, vl, wl};
    const T up_c = bup[c.q], dn_c = bdn[c.q];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int R[3] = {c.i, c.j, c.k};
        if (closed(g, a) && R[a] == extent(g, a) - 1) {
            lim[a][c.q] = T(0);
            continue;
        }
        R[a] += 1;
        const long long qr = at(g, R[0], R[1], R[2]);
        const T U = vel[a][c.q];
        const T up = min2(T(1), min2(dn_c, bup[qr]));
        const T dn = min2(T(1), min2(up_c, bdn[qr]));
        lim[a][c.q] = (pos_part(U) * up) + (neg_part(U) * dn);
    }
}

#pragma clang fp contract(on)

}  // namespace stages
}  // namespace mpdata
