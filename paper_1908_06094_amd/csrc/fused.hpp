// fused.hpp -- one MPDATA corrective pass as a single k-marching HIP kernel.
//
// A pass takes the iterate phi = psi^(m-1) and the previous pass's face
// velocities and produces psi^(m): antidiffusive pseudo-velocities, (if
// limited) the local bounds, the in/out flux sums and beta, the limited
// velocities and the donor-cell update with them.  Fusing these stages keeps
// every intermediate on chip: per cell the pass reads phi, psi^n, three face
// velocities and G once and writes psi^(m) (plus its limited velocities when
// another pass follows), which is the fusion-with-scratch-pad idea the paper
// applies to the upwind stages (Section 6.1, Table 2, Listing 9).
//
// Mapping onto gfx950:
//   * a workgroup is 16 waves of 64 lanes; lane = x, wave = y.  It owns a
//     60 x 12 interior tile plus a halo of 2 and marches up the k axis, so
//     each stage is computed once per column and plane (no halo recompute
//     along k);
//   * x neighbours come from DPP lane shifts (wave_shl / wave_shr), y
//     neighbours from one LDS plane slot per exchanged quantity, k neighbours
//     from the column's own register history;
//   * coalesced, i-fastest HBM rows of 64 elements per wave.
//
// Arithmetic differs from the scheme's literal order in one place: the
// antidiffusive velocity (|U| - U^2/Gf) A - (U/Gf)(Vb_1 B_1 + Vb_2 B_2),
// with A and B ratios over the pair sums, is evaluated over one common
// denominator (one IEEE division per face instead of four), and the two beta
// ratios of a cell share one division.  In FP64 this changes results by a few
// ulp.  In FP32 (where the product of three guarded denominators could
// underflow) the ratios are taken one by one.
#pragma once

#include "common.hpp"

namespace mpdata {
namespace fused {

constexpr int kLanes = 64;               // x extent of a tile, halo included
constexpr int kRows = 16;                // y extent (waves per workgroup)
constexpr int kHalo = 2;
constexpr int kTileX = kLanes - 2 * kHalo;   // 60 interior columns
constexpr int kTileY = kRows - 2 * kHalo;    // 12 interior rows
constexpr int kThreads = kLanes * kRows;     // 1024

// ---------------------------------------------------------------------------
// Lane shifts.  next(v): lane l receives lane l+1's value; prev(v): lane l-1's.
// The lane without a source receives 0 (it lies in the halo that the shrinking
// valid region discards).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false); }

__device__ __forceinline__ double lane_next(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(dpp_next_i(hi), dpp_next_i(lo));
}
__device__ __forceinline__ double lane_prev(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(dpp_prev_i(hi), dpp_prev_i(lo));
}
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_next_i(__float_as_int(v))); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_prev_i(__float_as_int(v))); }

// ---------------------------------------------------------------------------
// Antidiffusive velocity at one face from its ingredients:
//   n0/d0   the gradient ratio's numerator and guarded pair sum (+ side first)
//   n1/d1   the first transverse ratio (lower axis), n2/d2 the second
//   vs1/vs2 the sums of the four transverse face velocities (Vb = vs / 4)
//   gsum    G(left) + G(right) (Gf = gsum / 2), u the face velocity
// ---------------------------------------------------------------------------
__device__ __forceinline__ double antidiff_face(double n0, double d0, double n1, double d1, double n2, double d2,
                                                double vs1, double vs2, double gsum, double u)
{
    // (|u| - u^2/Gf) n0/d0 - (u/Gf)((vs1/4)(n1/(2 d1)) + (vs2/4)(n2/(2 d2)))
    //   = [(|u| gsum - 2u^2) n0 d1 d2 - (u/4) d0 (vs1 n1 d2 + vs2 n2 d1)] / (gsum d0 d1 d2)
    const double d12 = d1 * d2;
    const double au = u < 0.0 ? -u : u;
    const double t1 = ((au * gsum - 2.0 * (u * u)) * n0) * d12;
    const double t2 = (0.25 * u) * d0 * (vs1 * n1 * d2 + vs2 * n2 * d1);
    return (t1 - t2) / ((gsum * d0) * d12);
}

__device__ __forceinline__ float antidiff_face(float n0, float d0, float n1, float d1, float n2, float d2,
                                               float vs1, float vs2, float gsum, float u)
{
    const float A = __fdividef(n0, d0);
    const float B1 = 0.5f * __fdividef(n1, d1);
    const float B2 = 0.5f * __fdividef(n2, d2);
    const float rgf = __fdividef(2.0f, gsum);      // 1 / Gf
    const float au = u < 0.0f ? -u : u;
    return (au - (u * u) * rgf) * A - (u * rgf) * ((0.25f * vs1) * B1 + (0.25f * vs2) * B2);
}

// Limiter coefficients of one cell, the ratio taken in FP64 for both types.
template <class T>
__device__ __forceinline__ void beta_pair(T hi, T lo, T phi, T g, T fin, T fout, double eps, T& bup, T& bdn)
{
    const double a = (double)fin + eps;
    const double b = (double)fout + eps;
    const double r = 1.0 / (a * b);
    bup = (T)(((double)((hi - phi) * g) * b) * r);
    bdn = (T)(((double)((phi - lo) * g) * a) * r);
}

template <class T> __device__ __forceinline__ T min3(T a, T b, T c) { return min2(a, min2(b, c)); }

// Workgroup barrier ordering LDS only: prefetched global loads stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------
template <class T>
struct PassArgs {
    const T* phi;    // psi^(m-1)
    const T* psin;   // psi^n (limiter bounds)
    const T* u;      // previous pass's velocities (the Courant numbers for pass 2)
    const T* v;
    const T* w;      // may be NULL: all vertical velocities 0
    const T* g;
    T* out;          // psi^(m)
    T* ul;           // limited velocities (written when another pass follows)
    T* vl;
    T* wl;
    double eps;
    int tiles_x, tiles_y;
};

// Index along one axis for a virtual coordinate x (possibly outside [0, n)):
// periodic wraps, closed clamps.
__device__ __forceinline__ int map_index(int x, int n, int closed)
{
    if (closed) return x < 0 ? 0 : (x >= n ? n - 1 : x);
    int r = x % n;
    return r < 0 ? r + n : r;
}

// Is the face x+1/2 (virtual x) a closed wall or beyond one?
__device__ __forceinline__ bool wall_face(int x, int n, int closed) { return closed && (x < 0 || x >= n - 1); }

template <class T>
struct Slots {
    // y-exchange planes, one value per (row, lane)
    T phi[kRows][kLanes], u[kRows][kLanes], w[kRows][kLanes], g[kRows][kLanes];
    T px[kRows][kLanes], vpx[kRows][kLanes], pz[kRows][kLanes], vpz[kRows][kLanes];
    T mx[kRows][kLanes], mn[kRows][kLanes], fpy[kRows][kLanes], fmy[kRows][kLanes];
    T bup[kRows][kLanes], bdn[kRows][kLanes];
    T fy[2][kRows][kLanes];
};

template <class T, bool LIMIT, bool WRITE_VEL>
__global__ void __launch_bounds__(kThreads) k_pass(Geo geo, PassArgs<T> a)
{
    __shared__ Slots<T> S;

    const int lane = threadIdx.x & (kLanes - 1);
    const int row = threadIdx.x >> 6;
    const int up = row < kRows - 1 ? row + 1 : row;     // clamped: the edge rows are halo
    const int dn = row > 0 ? row - 1 : row;

    const int tile = blockIdx.x;
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int gi = tx * kTileX - kHalo + lane;           // virtual column of this lane
    const int gj = ty * kTileY - kHalo + row;
    const int ci = map_index(gi, geo.nx, geo.closed_x);
    const int cj = map_index(gj, geo.ny, geo.closed_y);
    const bool xwall = wall_face(gi, geo.nx, geo.closed_x);
    const bool ywall = wall_face(gj, geo.ny, geo.closed_y);
    const long long col = (long long)cj * geo.sy + ci;
    const bool writer = lane >= kHalo && lane < kLanes - kHalo && row >= kHalo && row < kRows - kHalo &&
                        gi < geo.nx && gj < geo.ny;

    const T eps = (T)a.eps;
    const T zero = T(0);

    // plane loader: cell quantities through the halo rule, faces masked at walls
    struct Plane {
        T phi, psin, u, v, w, g;
    };
    auto load = [&](int k) {
        Plane p;
        const int ck = map_index(k, geo.nz, geo.closed_z);
        const long long q = (long long)ck * geo.sz + col;
        p.phi = a.phi[q];
        p.psin = LIMIT ? a.psin[q] : zero;
        p.u = xwall ? zero : a.u[q];
        p.v = ywall ? zero : a.v[q];
        p.w = (a.w == nullptr || wall_face(k, geo.nz, geo.closed_z)) ? zero : a.w[q];
        p.g = a.g[q];
        return p;
    };

    // ---- register history of this column ----
    // plane k+1 ("n"), k ("c"), k-1 ("p"), where k = t-1 is the plane whose
    // antidiffusive velocities and beta are formed in march step t
    T phi_p = 0, phi_c = 0, phi_n = 0, nphi_c = 0, nphi_n = 0;
    T u_c = 0, u_n = 0, v_c = 0, v_n = 0, w_c = 0, w_n = 0;
    T g_p = 0, g_c = 0, g_n = 0, gx_c = 0, gx_n = 0;
    T px_p = 0, px_c = 0, px_n = 0, px_c_up = 0, px_c_dn = 0, px_n_up = 0, px_n_dn = 0;
    T py_p = 0, py_c = 0, py_n = 0;
    T phiup_c = 0, phiup_n = 0;
    T vpx_c = 0, vpx_n = 0, vpxdn_c = 0, vpxdn_n = 0;
    T wpx_p = 0, wpx_c = 0, wpx_n = 0, wpy_p = 0, wpy_c = 0, wpy_n = 0;
    T upy_c = 0, upy_n = 0, gpy_c = 0, gpy_n = 0;
    T mx_p = 0, mx_c = 0, mx_n = 0, mn_p = 0, mn_c = 0, mn_n = 0;
    T uz_p = 0;                 // antidiffusive velocity at face k-1/2
    T bup_p = 0, bdn_p = 0;     // beta at plane k-1
    T ulx_p = 0, uly_p = 0;     // limited x/y velocities at plane k-1
    T fx_p = 0, fy_p = 0;       // x and y fluxes at plane k-1
    T fz_pp = 0;                // z flux at face k-3/2

    const int kb = 0, ke = geo.nz;
    int par = 0;                // parity of the Fy slot written in this step

    Plane nx_ = load(kb - 3);
    for (int t = kb - 3; t <= ke + 1; ++t) {
        // ---------------- phase 0: plane t arrives ----------------
        const Plane pl = nx_;
        if (t + 1 <= ke + 1) nx_ = load(t + 1);     // prefetch the next plane

        // rotate: n -> c -> p
        phi_p = phi_c; phi_c = phi_n; phi_n = pl.phi;
        nphi_c = nphi_n; nphi_n = lane_next(pl.phi);
        u_c = u_n; u_n = pl.u;
        v_c = v_n; v_n = pl.v;
        w_c = w_n; w_n = pl.w;
        g_p = g_c; g_c = g_n; g_n = pl.g;
        gx_c = gx_n; gx_n = pl.g + lane_next(pl.g);
        px_p = px_c; px_c = px_n; px_n = nphi_n + pl.phi;
        px_c_up = px_n_up; px_c_dn = px_n_dn;
        py_p = py_c; py_c = py_n;
        phiup_c = phiup_n;
        vpx_c = vpx_n; vpx_n = pl.v + lane_next(pl.v);
        vpxdn_c = vpxdn_n;
        wpx_p = wpx_c; wpx_c = wpx_n; wpx_n = pl.w + lane_next(pl.w);
        wpy_p = wpy_c; wpy_c = wpy_n;
        upy_c = upy_n;
        gpy_c = gpy_n;
        if (LIMIT) {
            mx_p = mx_c; mx_c = mx_n; mx_n = max2(pl.psin, pl.phi);
            mn_p = mn_c; mn_c = mn_n; mn_n = min2(pl.psin, pl.phi);
        }
        const T pz_c = phi_n + phi_c;      // z face k+1/2: + side (k+1) first
        const T vpz_c = v_c + v_n;         // lower cell first
        const T upz_c = u_c + u_n;

        S.phi[row][lane] = pl.phi;
        S.u[row][lane] = pl.u;
        S.w[row][lane] = pl.w;
        S.g[row][lane] = pl.g;
        S.px[row][lane] = px_n;
        S.vpx[row][lane] = vpx_n;
        S.pz[row][lane] = pz_c;
        S.vpz[row][lane] = vpz_c;
        lds_barrier();

        // ---------------- phase 1: y neighbours of plane t, velocities of plane k ----------------
        phiup_n = S.phi[up][lane];
        py_n = phiup_n + pl.phi;
        upy_n = pl.u + S.u[up][lane];
        wpy_n = pl.w + S.w[up][lane];
        gpy_n = pl.g + S.g[up][lane];
        px_n_up = S.px[up][lane];
        px_n_dn = S.px[dn][lane];
        vpxdn_n = S.vpx[dn][lane];
        const T pz_up = S.pz[up][lane];
        const T pz_dn = S.pz[dn][lane];
        const T vpz_dn = S.vpz[dn][lane];

        // x face (i+1/2, j, k): transverse y then z
        const T ux = antidiff_face(nphi_c - phi_c, px_c + eps,
                                   px_c_up - px_c_dn, (px_c_up + px_c_dn) + eps,
                                   px_n - px_p, (px_n + px_p) + eps,
                                   vpx_c + vpxdn_c, wpx_c + wpx_p, gx_c, u_c);
        // y face (i, j+1/2, k): transverse x then z
        const T py_nx = lane_next(py_c), py_pv = lane_prev(py_c);
        const T uy = antidiff_face(phiup_c - phi_c, py_c + eps,
                                   py_nx - py_pv, (py_nx + py_pv) + eps,
                                   py_n - py_p, (py_n + py_p) + eps,
                                   upy_c + lane_prev(upy_c), wpy_c + wpy_p, gpy_c, v_c);
        // z face (i, j, k+1/2): transverse x then y
        const T pz_nx = lane_next(pz_c), pz_pv = lane_prev(pz_c);
        const T uz = antidiff_face(phi_n - phi_c, pz_c + eps,
                                   pz_nx - pz_pv, (pz_nx + pz_pv) + eps,
                                   pz_up - pz_dn, (pz_up + pz_dn) + eps,
                                   upz_c + lane_prev(upz_c), vpz_c + vpz_dn, g_c + g_n, w_c);

        T ulx, uly, ulz;       // limited velocities: x, y at plane k; z at face k-1/2
        if (LIMIT) {
            const T fpy = pos_part(uy) * phi_c;
            const T fmy = neg_part(uy) * phiup_c;
            S.mx[row][lane] = mx_c;
            S.mn[row][lane] = mn_c;
            S.fpy[row][lane] = fpy;
            S.fmy[row][lane] = fmy;
            lds_barrier();

            // ---------------- phase 2: bounds, in/out, beta at plane k ----------------
            T hi = max2(max2(mx_c, max2(lane_next(mx_c), lane_prev(mx_c))),
                        max2(max2(S.mx[up][lane], S.mx[dn][lane]), max2(mx_p, mx_n)));
            T lo = min2(min2(mn_c, min2(lane_next(mn_c), lane_prev(mn_c))),
                        min2(min2(S.mn[up][lane], S.mn[dn][lane]), min2(mn_p, mn_n)));
            const T fpx = pos_part(ux) * phi_c;
            const T fmx = neg_part(ux) * nphi_c;
            const T fpz = pos_part(uz) * phi_c;
            const T fmz = neg_part(uz) * phi_n;
            const T fpz_l = pos_part(uz_p) * phi_p;
            const T fmz_l = neg_part(uz_p) * phi_c;
            const T fin = ((lane_prev(fpx) - fmx) + (S.fpy[dn][lane] - fmy)) + (fpz_l - fmz);
            const T fout = ((fpx - lane_prev(fmx)) + (fpy - S.fmy[dn][lane])) + (fpz - fmz_l);
            T bup, bdn;
            beta_pair<T>(hi, lo, phi_c, g_c, fin, fout, a.eps, bup, bdn);
            S.bup[row][lane] = bup;
            S.bdn[row][lane] = bdn;
            lds_barrier();

            // ---------------- phase 3a: limited velocities ----------------
            const T bup_up = S.bup[up][lane], bdn_up = S.bdn[up][lane];
            ulx = pos_part(ux) * min3(T(1), bdn, lane_next(bup)) + neg_part(ux) * min3(T(1), bup, lane_next(bdn));
            uly = pos_part(uy) * min3(T(1), bdn, bup_up) + neg_part(uy) * min3(T(1), bup, bdn_up);
            ulz = pos_part(uz_p) * min3(T(1), bdn_p, bup) + neg_part(uz_p) * min3(T(1), bup_p, bdn);
            bup_p = bup;
            bdn_p = bdn;
        } else {
            ulx = ux;
            uly = uy;
            ulz = uz_p;
        }

        // ---------------- phase 3b: donor-cell update of plane k-1 ----------------
        const T fx_c = pos_part(ulx) * phi_c + neg_part(ulx) * nphi_c;
        const T fy_c = pos_part(uly) * phi_c + neg_part(uly) * phiup_c;
        S.fy[par][row][lane] = fy_c;
        const T fz_h = pos_part(ulz) * phi_p + neg_part(ulz) * phi_c;     // face k-1/2
        const T fy_p_dn = S.fy[par ^ 1][dn][lane];
        const T fx_p_l = lane_prev(fx_p);      // all lanes: DPP reads need every source lane active
        const int ko = t - 2;                  // plane k-1
        if (writer && ko >= kb && ko < ke) {
            const T div = ((fx_p - fx_p_l) + (fy_p - fy_p_dn)) + (fz_h - fz_pp);
            const long long q = (long long)ko * geo.sz + col;
            a.out[q] = phi_p - div / g_p;
            if (WRITE_VEL) {
                a.ul[q] = ulx_p;
                a.vl[q] = uly_p;
                a.wl[q] = ulz;                 // face (k-1)+1/2
            }
        }
        fz_pp = fz_h;
        fx_p = fx_c;
        fy_p = fy_c;
        ulx_p = ulx;
        uly_p = uly;
        uz_p = uz;
        par ^= 1;
        if (!LIMIT) lds_barrier();   // phase-0 slots are rewritten next; with the limiter the
                                     // phase-2 and phase-3 barriers already separate them
    }
}

}  // namespace fused
}  // namespace mpdata
