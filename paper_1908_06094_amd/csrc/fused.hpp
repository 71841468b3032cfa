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
//   * a workgroup is 12 waves (768 threads); lane = x, row = y.  In FP64 a
//     tile row is one wave of 64 lanes (64 x 12 tile, 60 x 8 interior); in
//     FP32 it is half a wave (32 x 24 tile, 28 x 20 interior).  The tile
//     carries a halo of 2 and marches up the k axis, so each stage is
//     computed once per column and plane (no halo recompute along k);
//   * LDS holds one plane slot per exchanged quantity (114 KB in FP64: one
//     workgroup per CU, 3 waves per SIMD, up to 168 VGPRs; 57 KB in FP32:
//     two workgroups per CU, 6 waves per SIMD, up to 80 VGPRs);
//   * persistent launch: the (tile, plane) space is cut into equal
//     contiguous ranges, one per workgroup, grouped by XCD;
//   * x neighbours come from DPP lane shifts (wave_shl / wave_shr), y
//     neighbours from the LDS slots, k neighbours from the column's own
//     register history;
//   * the next plane is prefetched one march step ahead with every load
//     unconditional, and a step's results are stored at the start of the
//     following step, before its prefetch, so that waiting for a prefetch
//     (vmcnt counts loads and stores in order) never waits for a store;
//   * coalesced, i-fastest HBM rows (512 B in FP64, 128 B in FP32);
//   * in FP64 each wave runs only the stages its tile row feeds (the halo
//     rows skip the update, the outer ones nearly everything: pass_rows).
//
// Arithmetic differs from the scheme's literal order in two places.  The
// antidiffusive velocity (|U| - U^2/Gf) A - (U/Gf)(Vb_1 B_1 + Vb_2 B_2),
// with A and B ratios over the pair sums, is evaluated over one common
// denominator (one division per face instead of four), and the two beta
// ratios of a cell share one division.  FP64 quotients come from the
// reciprocal with Newton refinement (div_nr, within an ulp of the IEEE
// quotient).  In FP64 this changes results by a few ulp.  In FP32 (where the
// product of three guarded denominators could underflow) the ratios are
// taken one by one, each from the hardware reciprocal (1 ulp), and the
// update's quotient from the reciprocal with one residual correction.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace mpdata {
namespace fused {

#ifndef MPDATA_ROW_LANES_F64
#define MPDATA_ROW_LANES_F64 64
#endif
#ifndef MPDATA_ROW_LANES_F32
#define MPDATA_ROW_LANES_F32 32
#endif
constexpr int kThreads = 768;                // 12 waves: 3 per SIMD, up to 168 VGPRs each
constexpr int kHalo = 2;

// Default tile row width per element type.
template <class T>
struct DefaultLanes {
    static constexpr int value = sizeof(T) == 8 ? MPDATA_ROW_LANES_F64 : MPDATA_ROW_LANES_F32;
};

// Tile shape: a tile row is L lanes wide (a wave holds 64 / L rows) and the
// workgroup's N threads (768 unless stated) hold `rows` rows.  The
// single-problem passes use the default width of their type; the batched
// passes are also compiled for the other widths, among which the autotuner
// picks.
template <class T, int L = DefaultLanes<T>::value, int N = kThreads>
struct Tile {
    static constexpr int threads = N;
    static constexpr int lanes = L;
    static constexpr int shift = lanes == 64 ? 6 : (lanes == 32 ? 5 : 4);
    static constexpr int rows = N / lanes;
    static constexpr int tile_x = lanes - 2 * kHalo;   // interior columns
    static constexpr int tile_y = rows - 2 * kHalo;    // interior rows
    // workgroups per CU: the FP32 tile's LDS (57 KB) and registers (<= 80)
    // let two share a CU (6 waves per SIMD); the FP64 tile needs 114 KB
    static constexpr int wgs_per_cu = sizeof(T) == 4 ? 2 : 1;
    static constexpr int waves_per_simd = wgs_per_cu * N / 256;
    // velocities handed between passes in the tile layout (FP32: its 112-byte
    // tile rows make the (nz, ny, nx) stores mostly partial cache lines; in
    // FP64 the 480-byte rows are not, and the tile layout measured slower).
    // The layout is that of the default FP32 tile; other widths hand their
    // velocities over as (nz, ny, nx) fields.
    static constexpr bool tiled_velocities = sizeof(T) == 4 && L == DefaultLanes<T>::value;
    static_assert((1 << shift) == lanes && lanes >= 16 && lanes <= 64, "a tile row is 16, 32 or 64 lanes");
    // The pass with the donor-cell pass folded in (DONOR).  FP64 widens its x
    // halo to 3 (58 interior columns), so that psi^(1) is needed on lanes
    // 1 .. 62 only and every donor-cell x flux comes from a lane shift: the
    // row-end lanes then need no extra loads (their registers are what the
    // 168-register budget lacks).  FP32 keeps the halo of 2 (its tile layout
    // of the velocities handed to the next pass is the 28 x 20 interior) and
    // loads the neighbours beyond the row ends; it runs one workgroup per
    // CU, where its registers fit without spilling.
    static constexpr int donor_halo_x = sizeof(T) == 8 ? 3 : 2;
    static constexpr int donor_tile_x = lanes - 2 * donor_halo_x;
    static constexpr int donor_wgs_per_cu = 1;
    static constexpr int donor_waves_per_simd = donor_wgs_per_cu * N / 256;
};

// Threads of the single-problem pass kernels: the FP32 donor-fused pass runs
// 1024 (a 32 x 32 tile, 28 x 28 interior, 4 waves per SIMD in its 128
// registers) where the others run 768; it hands its velocities over in the
// layout of the plain pass's 28 x 20 interior.
template <class T, bool DONOR>
struct PassThreads {
    static constexpr int value = DONOR && sizeof(T) == 4 ? 1024 : kThreads;
    using TL = Tile<T, DefaultLanes<T>::value, value>;
    static constexpr int waves_per_simd = DONOR ? TL::donor_waves_per_simd : TL::waves_per_simd;
};

// ---------------------------------------------------------------------------
// Lane shifts.  next(v): lane l receives lane l+1's value; prev(v): lane l-1's.
// The lane without a source reads 0 (bound_ctrl; it lies in the halo that the
// shrinking valid region discards), so the destination needs no initial value.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_next_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_prev_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }

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
// FP64 quotient from the hardware reciprocal refined by one Newton step and
// one residual correction on the quotient (Markstein's scheme): the Newton
// step squares the reciprocal's relative error, the correction squares the
// quotient's again, which leaves the rounding of the last step: within an
// ulp of the IEEE quotient, without the scaling and special-case steps of
// the IEEE division sequence.  Every denominator here is a normal positive
// number (pair sums guarded by eps, products of them, G).
__device__ __forceinline__ double div_nr(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    const double q = n * r;
    return __builtin_fma(r, __builtin_fma(-d, q, n), q);
}
// FP32 quotient from the hardware reciprocal (1 ulp) and one residual
// correction: within an ulp of the IEEE quotient, without the scaling and
// fix-up steps of the IEEE division sequence (every denominator is a normal
// positive number).
__device__ __forceinline__ float div_nr(float n, float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = n * r;
    return __builtin_fmaf(r, __builtin_fmaf(-d, q, n), q);
}

__device__ __forceinline__ double antidiff_face(double n0, double d0, double n1, double d1, double n2, double d2,
                                                double vs1, double vs2, double gsum, double u)
{
    // (|u| - u^2/Gf) n0/d0 - (u/Gf)((vs1/4)(n1/(2 d1)) + (vs2/4)(n2/(2 d2)))
    //   = [(|u| gsum - 2u^2) n0 d1 d2 - (u/4) d0 (vs1 n1 d2 + vs2 n2 d1)] / (gsum d0 d1 d2)
    const double d12 = d1 * d2;
    const double au = __builtin_fabs(u);   // |u| (+0 for u = -0: only the sign of a zero can differ)
    const double t1 = ((au * gsum - 2.0 * (u * u)) * n0) * d12;
    const double t2 = (0.25 * u) * d0 * (vs1 * n1 * d2 + vs2 * n2 * d1);
    return div_nr(t1 - t2, (gsum * d0) * d12);
}

__device__ __forceinline__ float antidiff_face(float n0, float d0, float n1, float d1, float n2, float d2,
                                               float vs1, float vs2, float gsum, float u)
{
    // the ratios from hardware reciprocals (1 ulp each; an IEEE division is
    // about ten instructions)
    const float A = n0 * __builtin_amdgcn_rcpf(d0);
    const float B1 = 0.5f * (n1 * __builtin_amdgcn_rcpf(d1));
    const float B2 = 0.5f * (n2 * __builtin_amdgcn_rcpf(d2));
    const float rgf = 2.0f * __builtin_amdgcn_rcpf(gsum);      // 1 / Gf
    const float au = __builtin_fabsf(u);
    return (au - (u * u) * rgf) * A - (u * rgf) * ((0.25f * vs1) * B1 + (0.25f * vs2) * B2);
}

// Limiter coefficients of one cell, the ratio taken in FP64 for both types.
template <class T>
__device__ __forceinline__ void beta_pair(T hi, T lo, T phi, T g, T fin, T fout, double eps, T& bup, T& bdn)
{
    const double a = (double)fin + eps;
    const double b = (double)fout + eps;
    const double r = div_nr(1.0, a * b);
    bup = (T)(((double)((hi - phi) * g) * b) * r);
    bdn = (T)(((double)((phi - lo) * g) * a) * r);
}


// [c]+ and [c]- as single v_max / v_min instructions (the sign of a zero
// result may differ from a compare-and-select; no value does)
__device__ __forceinline__ double pos_f(double c) { return __builtin_fmax(c, 0.0); }
__device__ __forceinline__ double neg_f(double c) { return __builtin_fmin(c, 0.0); }
__device__ __forceinline__ float pos_f(float c) { return __builtin_fmaxf(c, 0.0f); }
__device__ __forceinline__ float neg_f(float c) { return __builtin_fminf(c, 0.0f); }
__device__ __forceinline__ double fmx(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double fmn(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float fmx(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ float fmn(float a, float b) { return __builtin_fminf(a, b); }
template <class T> __device__ __forceinline__ T min3(T a, T b, T c) { return fmn(a, fmn(b, c)); }

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima): wait for
// every vector memory operation of this wave.
__device__ __forceinline__ void vmem_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

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
    T* ul;           // limited velocities (written when another pass follows),
    T* vl;           // in the tile layout
    T* wl;
    double eps;
    int tiles_x, tiles_y;
    int vel_tiled;   // u, v, w are in the tile layout (passes >= 3), else (nz, ny, nx)
    // What the recording kernels (REC, FP64, for the adjoint) also store, as
    // (nz, ny, nx) fields: the antidiffusive velocities and (with the
    // limiter) beta, clamped to at most 1 (min(1, beta) is all that the
    // limited velocities and their adjoint's branch choices read, and beta
    // only matters where it is below 1).
    T* rux;
    T* ruy;
    T* ruz;
    T* rbu;
    T* rbd;
    T* rphi;   // REC with DONOR: psi^(1), the input iterate the pass forms
};

// Tile layout of the limited velocities that one pass hands to the next
// (where Tile<T>::tiled_velocities; otherwise they are (nz, ny, nx) fields):
// for plane k, tile (tx, ty) (number ty * tiles_x + tx), interior row r and
// column c, element (k * tiles + tile) * tile_x * tile_y + r * tile_x + c.
// A tile writes its whole block of a plane in one march step, so its
// velocity stores fill cache lines instead of ending mid line at the tile's
// x edges.
template <class T>
__host__ __device__ inline long long tiled_plane(int tiles_x, int tiles_y)
{
    return (long long)tiles_x * tiles_y * Tile<T>::tile_x * Tile<T>::tile_y;
}
// Elements of one inter-pass velocity field for an nx x ny x nz grid.
template <class T>
__host__ __device__ inline long long vel_elems(int nx, int ny, int nz)
{
    if (!Tile<T>::tiled_velocities) return (long long)nx * ny * nz;
    const int tiles_x = (nx + Tile<T>::tile_x - 1) / Tile<T>::tile_x;
    const int tiles_y = (ny + Tile<T>::tile_y - 1) / Tile<T>::tile_y;
    return tiled_plane<T>(tiles_x, tiles_y) * nz;
}

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

template <class T, int L = DefaultLanes<T>::value, int N = kThreads>
struct Slots {
    static constexpr int kRows = Tile<T, L, N>::rows, kLanes = L, kThreads = N;
    // y-exchange planes, one value per (row, lane); phi, px and vpx keep the
    // last two planes (slot = plane parity) so that plane k's neighbours are
    // read one march step after they were published
    T phi[2][kRows][kLanes], px[2][kRows][kLanes], vpx[2][kRows][kLanes];
    T u[kRows][kLanes], w[kRows][kLanes], g[kRows][kLanes];
    T pz[kRows][kLanes], vpz[kRows][kLanes];
    T mx[kRows][kLanes], mn[kRows][kLanes], fpy[kRows][kLanes], fmy[kRows][kLanes];
    T bup[kRows][kLanes], bdn[kRows][kLanes];
    T fy[2][kRows][kLanes];
};

// The pass that also runs the donor-cell pass (DONOR) needs four more plane
// slots: psi^n and Cy of the current plane and of the next (rings by plane
// parity), published one march step ahead of their use, from which each row
// forms the donor-cell fluxes through its upper and its lower y face.
template <class T, int L = DefaultLanes<T>::value, int N = kThreads>
struct SlotsDonor : Slots<T, L, N> {
    T psd[2][Tile<T, L, N>::rows][L];
    T cyd[2][Tile<T, L, N>::rows][L];
};

// One column's values of one plane: the loaded fields and what is derived
// from them.  Three banks hold the planes k-1, k and k+1.
template <class T>
struct Bank {
    T phi, u, v, w, g;                     // loaded
    T px, py, vpx, wpx, wpy, upy, gpy;     // pair sums (see the face formulas)
    T mx, mn;                              // max / min of psi^n and phi
};
template <class T>
struct Raw {
    T phi, psin, u, v, w, g;
    // DONOR only: psi^n and Cx beyond the row's ends (lanes 0 and R-1), and
    // psi^n and Cy beyond the tile's outer rows (rows 0 and R-1)
    T xe, cxl, yx, cyd;
};

// March output planes [kb, ke) of one tile of one problem: the part of
// one wave, whose rows play role ROLE (all waves of the workgroup march
// together and meet at the same barriers).
//   ROLE 0: rows holding outputs; every stage.
//   ROLE 1: the second halo rows (1 and R-2 of R rows): with the limiter,
//           the face velocities, bounds and beta, which the neighbouring
//           output row's limited velocities need, and (row 1) the limited
//           y flux into row 2; without it, (row 1) the y velocity and flux.
//   ROLE 2: the outer halo rows (0 and R-1): their loads and LDS slots and,
//           with the limiter, (row 0) the y-face velocity below row 1,
//           which row 1's beta needs.
// DONOR: the pass is the first corrective pass of a step and forms its input
// iterate psi^(1) itself, by the donor-cell pass on psi^n with the Courant
// numbers (a.u, a.v, a.w), plane by plane ahead of its use (a.phi is not
// read).  psi^n and Cy are loaded one plane ahead of the other fields and
// published to LDS, so that each row forms the donor-cell fluxes through
// both of its y faces from its own and its neighbours' values without a
// further barrier; the row-end lanes and the outer rows load their
// neighbours beyond the tile.  Per cell the pass then reads psi^n, Cx, Cy,
// Cz and G once: the step's separate donor-cell pass and its psi^(1) round
// trip through HBM disappear.
template <class T, bool LIMIT, bool WRITE_VEL, int ROLE, bool REC, bool DONOR, class SL>
__device__ __forceinline__ void pass_rows(const Geo& geo, const PassArgs<T>& a, SL& S, const int tile,
                                          const int kb, const int ke)
{
    using TL = Tile<T, SL::kLanes, SL::kThreads>;
    constexpr int kLanes = TL::lanes, kRows = TL::rows;
    constexpr int kTileY = TL::tile_y;
    constexpr int kLayY = Tile<T, SL::kLanes>::tile_y;   // the tile layout's block height (the plain pass's)
    // x halo and interior width of this kernel (the donor-fused FP64 pass
    // widens its x halo); the tile layout of handed-over velocities keeps the
    // plain pass's interior
    constexpr int kHX = DONOR ? TL::donor_halo_x : kHalo;
    constexpr int kTileX = kLanes - 2 * kHX;
    constexpr int kLayX = TL::tile_x;
    constexpr bool kXEdgeLoads = DONOR && kHX == kHalo;   // row-end lanes load their outer neighbour
    const int lane = threadIdx.x & (kLanes - 1);
    const int row = threadIdx.x >> TL::shift;
    const int up = row < kRows - 1 ? row + 1 : row;     // clamped: the edge rows are halo
    const int dn = row > 0 ? row - 1 : row;
    const T eps = (T)a.eps;
    const T zero = T(0);
    {
        const int tx = tile % a.tiles_x;
        const int ty = tile / a.tiles_x;
        const int gi = tx * kTileX - kHX + lane;         // virtual column of this lane
        const int gj = ty * kTileY - kHalo + row;
        const int ci = map_index(gi, geo.nx, geo.closed_x);
        const int cj = map_index(gj, geo.ny, geo.closed_y);
        const bool xwall = wall_face(gi, geo.nx, geo.closed_x);
        const bool ywall = wall_face(gj, geo.ny, geo.closed_y);
        // a plane holds at most 2^30 cells (checked on the host): 32-bit offsets
        const unsigned col = (unsigned)(cj * (int)geo.sy + ci);
        const bool writer = lane >= kHX && lane < kLanes - kHX && row >= kHalo && row < kRows - kHalo &&
                            gi < geo.nx && gj < geo.ny;
        // this lane's cell in the tile layout of the velocities (blocks of
        // the plain pass's kLayX x kLayY interior)
        const int lay_tiles_x = (geo.nx + kLayX - 1) / kLayX;
        const int lay_tiles_y = (geo.ny + kLayY - 1) / kLayY;
        const int ttx = ci / kLayX, tty = cj / kLayY;
        const unsigned tcol = (unsigned)((tty * lay_tiles_x + ttx) * (kLayX * kLayY) +
                                         (cj - tty * kLayY) * kLayX + (ci - ttx * kLayX));
        const long long tplane = tiled_plane<T>(lay_tiles_x, lay_tiles_y);

        // plane loader: cell quantities through the halo rule.  Every load is
        // issued unconditionally and the wall masks are applied where the
        // plane is consumed (one march step later), so nothing waits for a
        // prefetch on the step that issues it.
        const bool has_w = a.w != nullptr;     // without w, g is loaded in its place and masked
        // DONOR: the neighbours beyond the row's ends and the tile's outer rows
        const bool x_lo = lane == 0, x_hi = lane == kLanes - 1;
        const bool y_lo = row == 0, y_hi = row == kRows - 1;
        // waves that may hold rows 0 and R-1: FP32 runs every wave in role 0,
        // and a wave of several rows takes the role of its innermost one
        constexpr bool kOuterRows = ROLE == 2 || sizeof(T) == 4 || kLanes < 64;
        const unsigned col_xe = (unsigned)(cj * (int)geo.sy + map_index(x_lo ? gi - 1 : gi + 1, geo.nx, geo.closed_x));
        const unsigned col_ye = (unsigned)(map_index(y_lo ? gj - 1 : gj + 1, geo.ny, geo.closed_y) * (int)geo.sy + ci);
        const bool xwall_l = wall_face(gi - 1, geo.nx, geo.closed_x);   // the face left of the cell
        const bool ywall_d = wall_face(gj - 1, geo.ny, geo.closed_y);   // the face below the cell
        // cells beyond a closed wall (the donor-cell pass gives them the
        // boundary cell's value): rows by their own row, lanes through the
        // lane holding the flux of the boundary cell's inner face
        const bool y_virtual = geo.closed_y && (gj < 0 || gj >= geo.ny);
        const int gi0 = tx * kTileX - kHX;   // lane 0's column
        const bool x_edge_tile = DONOR && geo.closed_x && (gi0 < 0 || gi0 + kLanes - 1 >= geo.nx);

        auto load = [&](int k, Raw<T>& B) __attribute__((always_inline)) {
            const int ck = map_index(k, geo.nz, geo.closed_z);
            const long long pl = (long long)ck * geo.sz;
            const long long q = pl + col;
            const long long qv = TL::tiled_velocities && a.vel_tiled ? (long long)ck * tplane + tcol : q;
            if (!DONOR) B.phi = a.phi[q];
            if (LIMIT && !DONOR) B.psin = a.psin[q];
            B.u = a.u[qv];
            B.w = *(has_w ? a.w + qv : a.g + q);
            B.g = a.g[q];
            if (DONOR) {
                // psi^n and Cy one plane ahead (the donor-cell pass of plane k
                // needs psi^n of k+1; Cy goes to LDS a step before its use)
                const long long q1 = (long long)map_index(k + 1, geo.nz, geo.closed_z) * geo.sz + col;
                B.psin = a.psin[q1];
                B.v = a.v[q1];
            } else {
                B.v = a.v[qv];
            }
            if (DONOR) {
                if (kXEdgeLoads) {
                    if (x_lo || x_hi) B.xe = a.psin[pl + col_xe];
                    if (x_lo) B.cxl = a.u[pl + col_xe];
                }
                if (kOuterRows) {
                    if (y_lo || y_hi) B.yx = a.psin[pl + col_ye];
                    if (y_lo) B.cyd = a.v[pl + col_ye];
                }
            }
        };

        // Stages this wave runs (see the row roles below).
        constexpr bool do_upd = ROLE == 0;
        constexpr bool do_fy = ROLE <= 1;
        constexpr bool do_beta = LIMIT && ROLE <= 1;
        constexpr bool do_uy = LIMIT || do_fy;
        constexpr bool do_uxz = LIMIT ? do_beta : do_upd;

        Bank<T> B0{}, B1{}, B2{};
        Raw<T> R{};
        T wsx = 0, wsy = 0;         // wpx and wpy summed over planes k and k-1
        T uz_p = 0;                 // antidiffusive velocity at face k-1/2
        T bup_p = 0, bdn_p = 0;     // beta at plane k-1
        T fx_p = 0, fy_p = 0;       // x and y fluxes at plane k-1
        T fz_pp = 0;                // z flux at face k-3/2
        T fz_d = 0;                 // DONOR: the donor-cell z flux at the face below the plane arriving next
        const int t_last = ke + 1;

        // Results of march step t (plane t-2 and the velocities of plane
        // t-1) are stored at the start of step t+1, before that step's
        // prefetch: waiting for a prefetch then never waits for a store.
        T st_upd = 0, st_ulz = 0, st_ulx = 0, st_uly = 0;
        auto flush = [&](const int t) __attribute__((always_inline)) {
            const int ko = t - 2;
            const long long q0 = (long long)ko * geo.sz + col;
            const long long v0 = (long long)ko * tplane + tcol;
            const long long w0 = TL::tiled_velocities ? v0 : q0;
            const long long wstep = TL::tiled_velocities ? tplane : geo.sz;
            if (writer && ko >= kb && ko < ke) {
                a.out[q0] = st_upd;
                if (WRITE_VEL) a.wl[w0] = st_ulz;     // face (k-1)+1/2
            }
            if (WRITE_VEL && writer && ko + 1 >= kb && ko + 1 < ke) {
                a.ul[w0 + wstep] = st_ulx;             // plane k
                a.vl[w0 + wstep] = st_uly;
            }
        };

        // March step t: plane t (bank N) has arrived; velocities and beta of
        // plane k = t-1 (bank C) are formed, and plane k-1 (bank P) is updated.
        // Step modes.  The first two steps of a segment only prime the
        // banks: plane kb-2 (loads, LDS slots, pair sums) and plane kb-1 (the
        // same, plus the z-face velocity above plane kb-2, which plane kb-1's
        // beta reads); from plane kb on, every stage runs.
        constexpr int kPrimeLoad = 0, kPrimeUz = 1, kFull = 2;
        auto step = [&](const int t, Bank<T>& P, Bank<T>& C, Bank<T>& N, auto mode_tag) __attribute__((always_inline)) {
            constexpr int kMode = decltype(mode_tag)::value;
            // the prefetch of plane t and the previous step's stores, both
            // issued one step ago, have landed: every later wait is free
            vmem_wait_all();
            flush(t - 1);
            // ---------------- DONOR: psi^(1) of plane t by the donor-cell pass ----------------
            T phi_t, psin_n, v_t;
            if constexpr (DONOR) {
                // plane t is the grid plane ck; virtual planes beyond a closed
                // top repeat plane nz-1, whose psi^(1) the previous step formed
                const int ck = map_index(t, geo.nz, geo.closed_z);
                const bool repeat_top = geo.closed_z && t >= geo.nz;
                const int sd = t & 1;
                // psi^n and Cy of plane ck, published one step ago; those of
                // plane t+1 for the next step
                const T p = S.psd[sd][row][lane];
                v_t = S.cyd[sd][row][lane];
                S.psd[sd ^ 1][row][lane] = R.psin;
                S.cyd[sd ^ 1][row][lane] = R.v;
                // the donor-cell flux through the upper y face of row r (the
                // same operands, in the same order, for every row that forms it)
                auto fy_row = [&](int r, int gr) __attribute__((always_inline)) {
                    const T vr = wall_face(gr, geo.ny, geo.closed_y) ? zero : S.cyd[sd][r][lane];
                    return pos_f(vr) * S.psd[sd][r][lane] + neg_f(vr) * S.psd[sd][r + 1][lane];
                };
                T fxr = zero, fyr = zero, fzr = zero;
                if (!repeat_top) {
                    const T U = xwall ? zero : R.u;
                    const T V = ywall ? zero : v_t;
                    const T W = (!has_w || wall_face(ck, geo.nz, geo.closed_z)) ? zero : R.w;
                    const T p_xn = lane_next(p);
                    const T p_xr = (kXEdgeLoads && x_hi) ? R.xe : p_xn;
                    const T p_yr = (kOuterRows && y_hi) ? R.yx : S.psd[sd][up][lane];
                    // below a closed bottom the plane repeats plane 0, whose upper
                    // neighbour is plane 1 (not the next virtual plane)
                    T p_zr = R.psin;
                    if (kMode != kFull && geo.closed_z && t < 0)
                        p_zr = a.psin[(long long)map_index(1, geo.nz, geo.closed_z) * geo.sz + col];
                    fxr = pos_f(U) * p + neg_f(U) * p_xr;
                    fyr = pos_f(V) * p + neg_f(V) * p_yr;
                    fzr = pos_f(W) * p + neg_f(W) * p_zr;
                    const T cxl = xwall_l ? zero : R.cxl;
                    const T fxl_n = lane_prev(fxr);
                    T fxl = (kXEdgeLoads && x_lo) ? pos_f(cxl) * R.xe + neg_f(cxl) * p : fxl_n;
                    T fyl;
                    if (kOuterRows && y_lo) {
                        const T cyd = ywall_d ? zero : R.cyd;
                        fyl = pos_f(cyd) * R.yx + neg_f(cyd) * p;
                    } else {
                        fyl = fy_row(dn, gj - 1);   // the row below's upper face
                    }
                    const T fzl = (geo.closed_z && ck == 0) ? zero : fz_d;
                    // A cell beyond a closed wall carries, by the halo rule,
                    // psi^(1) of the boundary cell it is clamped to: its loads
                    // are that cell's, and it takes that cell's pair of face
                    // fluxes (the wall face's is 0) in place of its own.
                    T fxr_c = fxr, fyr_c = fyr;
                    if (y_virtual) {
                        if (gj < 0) {
                            fyr_c = fy_row(row - gj, 0);
                            fyl = zero;
                        } else {
                            fyr_c = zero;
                            fyl = geo.ny >= 2 ? fy_row(row - (gj - (geo.ny - 2)), geo.ny - 2) : zero;
                        }
                    }
                    if (x_edge_tile) {   // uniform over the workgroup: the tile touches a closed x wall
                        const int wl = (int)(threadIdx.x & 63);
                        const int src = gi < 0 ? wl - gi : (gi >= geo.nx ? wl - (gi - (geo.nx >= 2 ? geo.nx - 2 : 0)) : wl);
                        const T f_src = __shfl(fxr, src, 64);
                        if (gi < 0) {
                            fxr_c = f_src;
                            fxl = zero;
                        } else if (gi >= geo.nx) {
                            fxr_c = zero;
                            fxl = geo.nx >= 2 ? f_src : zero;
                        }
                    }
                    phi_t = p - div_nr(((fxr_c - fxl) + (fyr_c - fyl)) + (fzr - fzl), R.g);
                    fz_d = fzr;
                    if (REC && writer && t >= kb && t < ke) a.rphi[(long long)t * geo.sz + col] = phi_t;
                } else {
                    phi_t = C.phi;
                }
                psin_n = p;
            } else {
                phi_t = R.phi;
                psin_n = R.psin;
                v_t = R.v;
            }
            // ---------------- phase 0: plane t arrives ----------------
            N.phi = phi_t;
            N.u = xwall ? zero : R.u;
            N.v = ywall ? zero : v_t;
            N.w = (!has_w || wall_face(t, geo.nz, geo.closed_z)) ? zero : R.w;
            N.g = R.g;
            load(t + 1 <= t_last ? t + 1 : t_last, R);   // prefetch the next plane (unconditionally)
            const int sn = t & 1, sc = sn ^ 1;      // ring slots of planes t (= k+1) and k
            N.px = lane_next(N.phi) + N.phi;
            N.vpx = N.v + lane_next(N.v);
            N.wpx = N.w + lane_next(N.w);
            if (LIMIT) {
                N.mx = fmx(psin_n, N.phi);
                N.mn = fmn(psin_n, N.phi);
            }
            const T pz_c = N.phi + C.phi;     // z face k+1/2: + side (k+1) first
            const T vpz_c = C.v + N.v;        // lower cell first
            const T upz_c = C.u + N.u;
            S.phi[sn][row][lane] = N.phi;
            S.u[row][lane] = N.u;
            S.w[row][lane] = N.w;
            S.g[row][lane] = N.g;
            S.px[sn][row][lane] = N.px;
            S.vpx[sn][row][lane] = N.vpx;
            S.pz[row][lane] = pz_c;
            S.vpz[row][lane] = vpz_c;
            lds_barrier();

            // ---------------- phase 1: y neighbours, antidiffusive velocities of plane k ----------------
            N.py = S.phi[sn][up][lane] + N.phi;
            N.upy = N.u + S.u[up][lane];
            N.wpy = N.w + S.w[up][lane];
            N.gpy = N.g + S.g[up][lane];
            const T phiup_c = S.phi[sc][up][lane];
            const T nphi_c = lane_next(C.phi);

            T ux = zero, uy = zero, uz = zero;
            if (do_uxz && kMode != kPrimeLoad) {
                const T px_c_up = S.px[sc][up][lane];
                const T px_c_dn = S.px[sc][dn][lane];
                const T vpxdn_c = S.vpx[sc][dn][lane];
                const T pz_up = S.pz[up][lane];
                const T pz_dn = S.pz[dn][lane];
                const T vpz_dn = S.vpz[dn][lane];
                const T gx_c = C.g + lane_next(C.g);
                // x face (i+1/2, j, k): transverse y then z
                if (kMode == kFull)
                    ux = antidiff_face(nphi_c - C.phi, C.px + eps,
                                       px_c_up - px_c_dn, (px_c_up + px_c_dn) + eps,
                                       N.px - P.px, (N.px + P.px) + eps,
                                       C.vpx + vpxdn_c, wsx, gx_c, C.u);
                // z face (i, j, k+1/2): transverse x then y
                const T pz_nx = lane_next(pz_c), pz_pv = lane_prev(pz_c);
                uz = antidiff_face(N.phi - C.phi, pz_c + eps,
                                   pz_nx - pz_pv, (pz_nx + pz_pv) + eps,
                                   pz_up - pz_dn, (pz_up + pz_dn) + eps,
                                   upz_c + lane_prev(upz_c), vpz_c + vpz_dn, C.g + N.g, C.w);
            }
            if (kMode != kFull) {
                if (kMode == kPrimeUz && do_uxz) uz_p = uz;
                wsx = N.wpx + C.wpx;
                wsy = N.wpy + C.wpy;
                lds_barrier();   // the next step rewrites the slots read above
                return;
            }
            if (do_uy) {
                // y face (i, j+1/2, k): transverse x then z
                const T py_nx = lane_next(C.py), py_pv = lane_prev(C.py);
                uy = antidiff_face(phiup_c - C.phi, C.py + eps,
                                   py_nx - py_pv, (py_nx + py_pv) + eps,
                                   N.py - P.py, (N.py + P.py) + eps,
                                   C.upy + lane_prev(C.upy), wsy, C.gpy, C.v);
            }

            // recording: the antidiffusive velocities of plane k (stored at
            // once: these stores follow this step's prefetch)
            const int kc = t - 1;
            const bool rec_here = REC && writer && kc >= kb && kc < ke;
            const long long qc = (long long)kc * geo.sz + col;
            if (REC && rec_here) {
                a.rux[qc] = ux;
                a.ruy[qc] = uy;
                a.ruz[qc] = uz;
            }

            // limited velocities: x, y at plane k; z at face k-1/2
            T ulx = ux, uly = uy, ulz = uz_p;
            if (LIMIT) {
                T fpy = zero, fmy = zero;
                if (do_uy) {
                    fpy = pos_f(uy) * C.phi;
                    fmy = neg_f(uy) * phiup_c;
                    S.fpy[row][lane] = fpy;
                    S.fmy[row][lane] = fmy;
                }
                S.mx[row][lane] = C.mx;
                S.mn[row][lane] = C.mn;
                lds_barrier();

                // ---------------- phase 2: bounds, in/out, beta at plane k ----------------
                T bup = zero, bdn = zero;
                if (do_beta) {
                    const T hi = fmx(fmx(C.mx, fmx(lane_next(C.mx), lane_prev(C.mx))),
                                     fmx(fmx(S.mx[up][lane], S.mx[dn][lane]), fmx(P.mx, N.mx)));
                    const T lo = fmn(fmn(C.mn, fmn(lane_next(C.mn), lane_prev(C.mn))),
                                     fmn(fmn(S.mn[up][lane], S.mn[dn][lane]), fmn(P.mn, N.mn)));
                    const T fpx = pos_f(ux) * C.phi;
                    const T fmx_ = neg_f(ux) * nphi_c;
                    const T fpz = pos_f(uz) * C.phi;
                    const T fmz = neg_f(uz) * N.phi;
                    const T fpz_l = pos_f(uz_p) * P.phi;
                    const T fmz_l = neg_f(uz_p) * C.phi;
                    const T fin = ((lane_prev(fpx) - fmx_) + (S.fpy[dn][lane] - fmy)) + (fpz_l - fmz);
                    const T fout = ((fpx - lane_prev(fmx_)) + (fpy - S.fmy[dn][lane])) + (fpz - fmz_l);
                    beta_pair<T>(hi, lo, C.phi, C.g, fin, fout, a.eps, bup, bdn);
                    // only min(1, beta) is ever used.  FP64 clamps once per cell
                    // (min(1, a, b) = min(min(1, a), min(1, b)) exactly) and
                    // keeps one min per use; FP32 has a three-operand min.
                    if (sizeof(T) == 8) {
                        bup = fmn(T(1), bup);
                        bdn = fmn(T(1), bdn);
                    }
                    S.bup[row][lane] = bup;
                    S.bdn[row][lane] = bdn;
                    if (REC && rec_here) {
                        a.rbu[qc] = bup;
                        a.rbd[qc] = bdn;
                    }
                }
                auto lim = [](T x, T y) __attribute__((always_inline)) {
                    return sizeof(T) == 8 ? fmn(x, y) : min3(T(1), x, y);
                };
                lds_barrier();

                // ---------------- phase 3a: limited velocities ----------------
                if (do_fy) {
                    const T bup_up = S.bup[up][lane], bdn_up = S.bdn[up][lane];
                    uly = pos_f(uy) * lim(bdn, bup_up) + neg_f(uy) * lim(bup, bdn_up);
                }
                if (do_upd) {
                    ulx = pos_f(ux) * lim(bdn, lane_next(bup)) + neg_f(ux) * lim(bup, lane_next(bdn));
                    ulz = pos_f(uz_p) * lim(bdn_p, bup) + neg_f(uz_p) * lim(bup_p, bdn);
                    bup_p = bup;
                    bdn_p = bdn;
                }
            }

            // ---------------- phase 3b: donor-cell update of plane k-1 ----------------
            const int par = t & 1;
            if (do_fy) {
                const T fy_c = pos_f(uly) * C.phi + neg_f(uly) * phiup_c;
                S.fy[par][row][lane] = fy_c;
                if (do_upd) {
                    const T fx_c = pos_f(ulx) * C.phi + neg_f(ulx) * nphi_c;
                    const T fz_h = pos_f(ulz) * P.phi + neg_f(ulz) * C.phi;     // face k-1/2
                    const T fy_p_dn = S.fy[par ^ 1][dn][lane];
                    const T fx_p_l = lane_prev(fx_p);      // every lane of the wave: DPP reads its neighbours
                    const T div = ((fx_p - fx_p_l) + (fy_p - fy_p_dn)) + (fz_h - fz_pp);
                    st_upd = P.phi - div_nr(div, P.g);     // plane k-1, stored by the next step
                    st_ulz = ulz;
                    st_ulx = ulx;
                    st_uly = uly;
                    fz_pp = fz_h;
                    fx_p = fx_c;
                    fy_p = fy_c;
                }
            }
            if (do_uxz) uz_p = uz;
            wsx = N.wpx + C.wpx;
            wsy = N.wpy + C.wpy;
            if (!LIMIT) lds_barrier();   // phase-0 slots are rewritten next; with the limiter the
                                         // phase-2 and phase-3 barriers already separate them
        };

        if constexpr (DONOR) {
            // psi^n of the first plane into its slot, and the donor-cell z
            // flux through the face below it (0 at a closed bottom)
            const int t0 = kb - 2;
            const int c0 = map_index(t0, geo.nz, geo.closed_z);
            const T p0 = a.psin[(long long)c0 * geo.sz + col];
            S.psd[t0 & 1][row][lane] = p0;
            S.cyd[t0 & 1][row][lane] = a.v[(long long)c0 * geo.sz + col];
            fz_d = zero;
            if (!(geo.closed_z && c0 == 0)) {
                const int cm = map_index(c0 - 1, geo.nz, geo.closed_z);
                const T pm = a.psin[(long long)cm * geo.sz + col];
                const T wm = has_w ? a.w[(long long)cm * geo.sz + col] : zero;
                fz_d = pos_f(wm) * pm + neg_f(wm) * p0;
            }
            lds_barrier();
        }
        load(kb - 2, R);
        step(kb - 2, B0, B1, B2, std::integral_constant<int, kPrimeLoad>{});
        B0 = B1;
        B1 = B2;
        step(kb - 1, B0, B1, B2, std::integral_constant<int, kPrimeUz>{});
        B0 = B1;
        B1 = B2;
        for (int t = kb; t <= t_last; ++t) {
            step(t, B0, B1, B2, std::integral_constant<int, kFull>{});
            B0 = B1;
            B1 = B2;
        }
        flush(t_last);
        lds_barrier();   // the next segment rewrites every slot
    }
}

// One tile's march, each wave in the role of its rows (a wave holding
// several rows takes the role of the row that needs most).  FP32 runs every
// wave in role 0: there only two waves of twelve hold no output row, and
// the kernel with three loop bodies spills more of its 80 registers.
template <class T, bool LIMIT, bool WRITE_VEL, bool REC = false, bool DONOR = false, class SL>
__device__ __forceinline__ void pass_segment(const Geo& geo, const PassArgs<T>& a, SL& S, const int tile,
                                             const int kb, const int ke)
{
    constexpr int kRows = SL::kRows, kRowsPerWave = 64 / SL::kLanes;
    static_assert(kHalo == 2, "the row roles assume a halo of 2");
    if (sizeof(T) == 4) {
        pass_rows<T, LIMIT, WRITE_VEL, 0, REC, DONOR>(geo, a, S, tile, kb, ke);
        return;
    }
    const int r_lo = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6) * kRowsPerWave);
    const int r_hi = r_lo + kRowsPerWave - 1;
    if (r_lo <= kRows - 3 && r_hi >= 2)
        pass_rows<T, LIMIT, WRITE_VEL, 0, REC, DONOR>(geo, a, S, tile, kb, ke);
    else if (r_lo <= kRows - 2 && r_hi >= 1)
        pass_rows<T, LIMIT, WRITE_VEL, 1, REC, DONOR>(geo, a, S, tile, kb, ke);
    else
        pass_rows<T, LIMIT, WRITE_VEL, 2, REC, DONOR>(geo, a, S, tile, kb, ke);
}

// Slots of a pass kernel (the donor-fused pass needs three more planes).
template <class T, bool DONOR, int L = DefaultLanes<T>::value, int N = kThreads>
using PassSlots = typename std::conditional<DONOR, SlotsDonor<T, L, N>, Slots<T, L, N>>::type;

// Logical workgroup id: the dispatcher deals workgroups round-robin over the
// 8 XCDs; consecutive logical ids (hence neighbouring work) share one XCD.
__device__ __forceinline__ int xcd_grouped_id()
{
    const int nwg = gridDim.x;   // a multiple of 8
    return (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
}

// One corrective pass of one problem.  Work split: the (tile, output plane)
// pairs in tile-major order are cut into equal contiguous ranges, one per
// workgroup, so every workgroup marches the same number of planes (a range
// may span a tile boundary).
template <class T, bool LIMIT, bool WRITE_VEL, bool REC = false, bool DONOR = false>
__global__ void __launch_bounds__((PassThreads<T, DONOR>::value), (PassThreads<T, DONOR>::waves_per_simd))
    k_pass(Geo geo, PassArgs<T> a)
{
    __shared__ PassSlots<T, DONOR, DefaultLanes<T>::value, PassThreads<T, DONOR>::value> S;
    const int nwg = gridDim.x;
    const int wg = xcd_grouped_id();
    const long long total = (long long)a.tiles_x * a.tiles_y * geo.nz;
    const long long span = (total + nwg - 1) / nwg;
    long long w0 = (long long)wg * span;
    const long long w1 = w0 + span < total ? w0 + span : total;
    while (w0 < w1) {
        const int tile = (int)(w0 / geo.nz);
        const int kb = (int)(w0 - (long long)tile * geo.nz);
        const int ke = (int)((long long)kb + (w1 - w0) < geo.nz ? kb + (w1 - w0) : geo.nz);
        w0 += ke - kb;
        pass_segment<T, LIMIT, WRITE_VEL, REC, DONOR>(geo, a, S, tile, kb, ke);
    }
}

// ---------------------------------------------------------------------------
// Batched passes: many problems (and tracers) in one launch.  Entry e covers
// work units [begin, begin + tiles * tracers * nz) in the order (tile,
// tracer, plane), so that the tracers of one tile, which share winds and G,
// run on neighbouring workgroups of one XCD and share its L2.
// ---------------------------------------------------------------------------
template <class T>
struct BatchEntry {
    Geo geo;
    PassArgs<T> args;        // tracer 0's fields; tracer t adds t * tracer_stride
    long long begin;         // first work unit
    long long tracer_stride; // elements between consecutive tracers' fields
    long long vel_stride;    // the same for the (tile-layout) velocity fields
    int tracers;
    int vel_per_tracer;      // previous velocities are per tracer (passes >= 3)
};

// N threads per workgroup (768: 12 waves; 1024: 16 waves, the tile
// 1024 / L rows tall).  WAVES_PER_SIMD: 3 = one 768-thread workgroup per CU
// (up to 168 VGPRs per wave); 6 = two (the FP32 kernel's LDS allows it;
// VGPRs <= 80); 4 = one 1024-thread workgroup (VGPRs <= 128).
template <class T, bool LIMIT, bool WRITE_VEL, int WAVES_PER_SIMD, bool DONOR = false, int L = DefaultLanes<T>::value,
          int N = kThreads>
__global__ void __launch_bounds__(N, WAVES_PER_SIMD) k_pass_batched(const BatchEntry<T>* __restrict__ tab,
                                                                    int n_entries, long long total)
{
    __shared__ PassSlots<T, DONOR, L, N> S;
    const int nwg = gridDim.x;
    const int wg = xcd_grouped_id();
    const long long span = (total + nwg - 1) / nwg;
    long long w0 = (long long)wg * span;
    const long long w1 = w0 + span < total ? w0 + span : total;
    while (w0 < w1) {
        // the entry holding w0 (binary search on the begin offsets)
        int lo = 0, hi = n_entries - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[mid].begin <= w0) lo = mid; else hi = mid - 1;
        }
        const BatchEntry<T>& e = tab[lo];
        const long long r = w0 - e.begin;
        const long long per_tile = (long long)e.tracers * e.geo.nz;
        const int tile = (int)(r / per_tile);
        const long long rr = r - (long long)tile * per_tile;
        const int tracer = (int)(rr / e.geo.nz);
        const int kb = (int)(rr - (long long)tracer * e.geo.nz);
        const int ke = (int)((long long)kb + (w1 - w0) < e.geo.nz ? kb + (w1 - w0) : e.geo.nz);
        w0 += ke - kb;
        PassArgs<T> a = e.args;
        const long long off = (long long)tracer * e.tracer_stride;
        if (!DONOR) a.phi += off;   // the donor-fused pass reads no iterate
        a.psin += off;
        a.out += off;
        const long long voff = (long long)tracer * e.vel_stride;
        if (e.vel_per_tracer) {
            a.u += voff;
            a.v += voff;
            if (a.w) a.w += voff;
        }
        if (WRITE_VEL) {
            a.ul += voff;
            a.vl += voff;
            a.wl += voff;
        }
        pass_segment<T, LIMIT, WRITE_VEL, false, DONOR>(e.geo, a, S, tile, kb, ke);
    }
}

}  // namespace fused
}  // namespace mpdata
