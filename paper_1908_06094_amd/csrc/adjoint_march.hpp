// adjoint_march.hpp -- the antidiffusive-velocity adjoint of a limited pass
// as one k-marching kernel (FP64).
//
// k_adj_inout_bounds_antidiff1 evaluates, per face, the partial derivatives
// of the antidiffusive velocity times the face's adjoint (seven "slot" values
// per face, adjoint.hpp) and k_adj_antidiff2 gathers them per cell; between
// the two, 21 slot fields go through HBM.  Here one kernel does both: a
// workgroup holds a tile of 32 x 16 columns (halo 1 in x and y) and marches
// up k.  Each step evaluates the first kernel's work for one plane of the
// tile (every column, halo included) and gathers the plane below for the
// interior columns from the slots the tile has put in its LDS (two planes)
// and those the column keeps in registers.  The
// gathers are the fast path of k_adj_antidiff2, term for term and in its
// order, so the results equal the two-kernel form bit for bit.  A pair of
// slots that the fast path adds as one sum and that lie in one column (a
// z-face's slot at planes k and k-1) is added once, by that column.
//
// Cells within two of a closed end (or on a periodic axis of fewer than four
// cells) take k_adj_antidiff2's general path: for them, and for every face
// that path reads (within three of a closed end), this kernel stores the
// slots and its partial results to HBM, and k_adj_antidiff2 (general cells
// only) gathers them afterwards.
#pragma once

#include "adjoint.hpp"
#include "fused.hpp"

namespace mpdata {
namespace adj {

#pragma clang fp contract(off)

constexpr int kMLanes = 32;                   // tile row width (x); two rows per wave
constexpr int kMRows = 16;                    // tile rows (y)
constexpr int kMThreads = kMLanes * kMRows;   // 512
constexpr int kMTileX = kMLanes - 2;          // interior columns
constexpr int kMTileY = kMRows - 2;           // interior rows

struct MarchArgs {
    double eps;
    const double* phi;                   // the pass's input iterate
    const double *ut, *vt, *wt;          // its antidiffusive velocities
    const double *lin, *lout, *lmx, *lmn;
    const unsigned char* code;           // the bounds' extremal entries
    const double *lutx, *luty, *lutz;    // the antidiffusive velocities' adjoint (limiter part)
    const double *pu, *pv, *pw;          // the pass's input velocities
    const double* gm;
    double* lpsin;                       // = when assign_psin, else +=
    double* slots;                       // 3 x kSlots fields of `field` elements
    long long field;
    double* lphi;                        // in: the donor-cell and limiter terms; out: dJ/dphi
    double *lu, *lv, *lw;                // the input velocities' adjoint (= when assign_vel, else +=)
    int assign_psin, assign_vel;
    int tiles_x, tiles_y;
};

// The LDS: a plane's slot values that the gathers of that plane and of the
// plane below read, in two buffers (by plane parity), and the y-face slot 3
// of the plane below the gathered one.
enum {
    Q00, Q01, Q02, Q04, Q05, Q06,   // x-face slots
    Q10, Q11, Q12, Q14, Q15, Q16,   // y-face slots
    QZ1, QZ2, QZ3, QZ4, QZ5, QZ6,   // z-face slots 1 .. 6 of the plane and the plane below, summed
    kMBuf
};
struct MarchLds {
    double b[2][kMBuf][kMRows][kMLanes];   // 144 KB
    double p13[kMRows][kMLanes];           // 4 KB
};

// Whether the cell takes k_adj_antidiff2's fast path (every axis periodic
// with >= 4 cells, or the cell >= 2 away from a closed end).
__device__ __forceinline__ bool gather_fast(const Geo& g, int i, int j, int k)
{
    const int c[3] = {i, j, k};
    bool f = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int n = extent(g, b);
        f = f && (closed(g, b) ? (c[b] >= 2 && c[b] <= n - 3) : n >= 4);
    }
    return f;
}

// Whether a general-path cell may read the slots of the cell's faces.
__device__ __forceinline__ bool slots_read_by_general(const Geo& g, int i, int j, int k)
{
    const int c[3] = {i, j, k};
    bool r = false;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int n = extent(g, b);
        r = r || (closed(g, b) ? (c[b] <= 2 || c[b] >= n - 3) : n < 4);
    }
    return r;
}

// What a column keeps from the planes below for the gathers: the slots that
// no other column reads (x-face 3, y-face 3 and z-face 0 of planes m-1 and
// m-2; z-face 1 .. 6 of plane m-1, to pair with plane m's) and the cell's
// values before the gather.
struct MarchCarry {
    double s03[2], s13[2], s20[2];   // [0]: plane m-1, [1]: plane m-2
    double s2[6];
    double lphi, tv[3];
};

// The first kernel's work at one cell (k_adj_inout_bounds_antidiff1, the same
// expressions in the same order).  The slots of the cell's three faces (0 at
// a closed wall) go to the LDS buffer of the plane (B); lpsin is stored when
// `out` (the cell is an output of this workgroup); the slots, dJ/dphi and the
// velocity adjoints go to HBM when `direct` (a general-path cell), the slots
// alone when `keep_slots`; otherwise dJ/dphi and the velocity adjoints before
// the gather stay in the carry.
__device__ __forceinline__ void march_b(const Geo& g, const Cell& c, const MarchArgs& a, bool out, bool direct,
                                        bool keep_slots, double (&B)[kMBuf][kMRows][kMLanes], int row, int lane,
                                        MarchCarry& h)
{
    double dl[3];
    const double acc = adj_inout_cell(g, c, a.phi, a.ut, a.vt, a.wt, a.lin, a.lout, dl);
    double gp, gf;
    adj_bounds_cell(g, c, a.code, a.lmx, a.lmn, gp, gf);
    if (out) {
        if (a.assign_psin) a.lpsin[c.q] = gp;
        else a.lpsin[c.q] += gp;
    }
    const double lam[3] = {a.lutx[c.q] + dl[0], a.luty[c.q] + dl[1], a.lutz[c.q] + dl[2]};
    const double* const vel[3] = {a.pu, a.pv, a.pw};
    double* lvel[3] = {a.lu, a.lv, a.lw};
    double own = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double s[kSlots], ldu = 0.0, own_a = 0.0;
        h.tv[ax] = 0.0;
        if (!antidiff1_face(g, c, ax, a.eps, a.phi, vel, a.gm, lam[ax], s, ldu, own_a)) {
#pragma unroll
            for (int e = 0; e < kSlots; ++e) s[e] = 0.0;
            if (direct && lvel[ax] && a.assign_vel) lvel[ax][c.q] = 0.0;   // a closed wall's unused slot
        } else {
            own += own_a;
            if (out && lvel[ax]) h.tv[ax] = a.assign_vel ? ldu : lvel[ax][c.q] + ldu;
            if (direct && lvel[ax]) lvel[ax][c.q] = h.tv[ax];
        }
        if (direct || keep_slots) {
            double* sp = a.slots + (long long)ax * kSlots * a.field + c.q;
#pragma unroll
            for (int e = 0; e < kSlots; ++e) sp[e * a.field] = s[e];
        }
        if (ax == 0) {
            B[Q00][row][lane] = s[0];
            B[Q01][row][lane] = s[1];
            B[Q02][row][lane] = s[2];
            B[Q04][row][lane] = s[4];
            B[Q05][row][lane] = s[5];
            B[Q06][row][lane] = s[6];
            h.s03[0] = s[3];
        } else if (ax == 1) {
            B[Q10][row][lane] = s[0];
            B[Q11][row][lane] = s[1];
            B[Q12][row][lane] = s[2];
            B[Q14][row][lane] = s[4];
            B[Q15][row][lane] = s[5];
            B[Q16][row][lane] = s[6];
            h.s13[0] = s[3];
        } else {
            h.s20[0] = s[0];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                B[QZ1 + e][row][lane] = s[e + 1] + h.s2[e];   // this plane's slot, then the plane below's
                h.s2[e] = s[e + 1];
            }
        }
    }
    h.lphi = 0.0;
    if (out) {
        h.lphi = (a.lphi[c.q] + (acc + gf)) + own;
        if (direct) a.lphi[c.q] = h.lphi;
    }
}

using fused::lane_prev;
using fused::lds_barrier;

// One tile's planes [kb, ke): march m = kb-1 .. ke, evaluating the first
// kernel's work at plane m and, from m = kb+1 on, gathering plane m-1 (the
// fast path of k_adj_antidiff2, term for term and in its order).
__device__ __forceinline__ void march_segment(const Geo& g, const MarchArgs& a, MarchLds& S, int tile, int kb,
                                              int ke)
{
    const int lane = threadIdx.x & (kMLanes - 1), row = threadIdx.x / kMLanes;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int gi = tx * kMTileX - 1 + lane, gj = ty * kMTileY - 1 + row;
    const bool inner = lane >= 1 && lane <= kMLanes - 2 && row >= 1 && row <= kMRows - 2 && gi < g.nx && gj < g.ny;
    // the column's cell after the halo rule; columns beyond the first one
    // past the domain's end feed no output and take the last column
    const int ci = gi > g.nx ? g.nx - 1 : nbr(gi, g.nx, g.closed_x);
    const int cj = gj > g.ny ? g.ny - 1 : nbr(gj, g.ny, g.closed_y);

    MarchCarry h;
#pragma unroll
    for (int e = 0; e < 2; ++e) h.s03[e] = h.s13[e] = h.s20[e] = 0.0;
#pragma unroll
    for (int e = 0; e < 6; ++e) h.s2[e] = 0.0;
    double lphi_k = 0.0, tv_k[3] = {0.0, 0.0, 0.0};
    bool gather_k = false;
    long long q_k = 0;

    for (int m = kb - 1; m <= ke; ++m) {
        Cell c;
        c.i = ci;
        c.j = cj;
        c.k = nbr(m, g.nz, g.closed_z);
        c.q = (long long)c.k * g.sz + (long long)c.j * g.sy + c.i;
        const bool out = inner && m >= kb && m < ke;
        const bool fast = out && gather_fast(g, c.i, c.j, c.k);
        const bool keep = out && slots_read_by_general(g, c.i, c.j, c.k);
        // plane m-2's slots that the gather of plane m-1 reads
        const double k1_s03 = h.s03[1], k1_s13 = h.s13[1], k1_s20 = h.s20[1];
        const double x03 = lane_prev(k1_s03);   // the left column's
        h.s03[1] = h.s03[0];
        h.s13[1] = h.s13[0];
        h.s20[1] = h.s20[0];
        lds_barrier();   // the previous step's gather has read the buffer written below
        S.p13[row][lane] = k1_s13;
        march_b(g, c, a, out, out && !fast, keep, S.b[m & 1], row, lane, h);
        lds_barrier();
        if (m >= kb + 1 && gather_k) {
            // gather plane k = m - 1: K = its buffer, N = plane m's
            const double(&K)[kMBuf][kMRows][kMLanes] = S.b[(m - 1) & 1];
            const double(&N)[kMBuf][kMRows][kMLanes] = S.b[m & 1];
            const int rd = row - 1, ru = row + 1, lp = lane - 1, ln = lane + 1;
            double acc = 0.0;
            // x faces
            acc += K[Q00][row][lp];
            acc += K[Q01][rd][lane] + K[Q01][rd][lp];
            acc += K[Q02][ru][lane] + K[Q02][ru][lp];
            acc += k1_s03 + x03;
            acc += N[Q04][row][lane] + N[Q04][row][lp];
            // y faces
            acc += K[Q10][rd][lane];
            acc += K[Q11][row][lp] + K[Q11][rd][lp];
            acc += K[Q12][row][ln] + K[Q12][rd][ln];
            acc += k1_s13 + S.p13[rd][lane];
            acc += N[Q14][row][lane] + N[Q14][rd][lane];
            // z faces
            acc += k1_s20;
            acc += K[QZ1][row][lp];
            acc += K[QZ2][row][ln];
            acc += K[QZ3][rd][lane];
            acc += K[QZ4][ru][lane];
            a.lphi[q_k] = lphi_k + acc;
            if (a.lu) {
                double accv = 0.0;
                accv += (K[Q15][row][lane] + K[Q15][rd][lane]) + (K[Q15][row][ln] + K[Q15][rd][ln]);
                accv += K[QZ5][row][lane] + K[QZ5][row][ln];
                a.lu[q_k] = tv_k[0] + accv;
            }
            if (a.lv) {
                double accv = 0.0;
                accv += (K[Q05][row][lane] + K[Q05][row][lp]) + (K[Q05][ru][lane] + K[Q05][ru][lp]);
                accv += K[QZ6][row][lane] + K[QZ6][ru][lane];
                a.lv[q_k] = tv_k[1] + accv;
            }
            if (a.lw) {
                double accv = 0.0;
                accv += (K[Q06][row][lane] + K[Q06][row][lp]) + (N[Q06][row][lane] + N[Q06][row][lp]);
                accv += (K[Q16][row][lane] + K[Q16][rd][lane]) + (N[Q16][row][lane] + N[Q16][rd][lane]);
                a.lw[q_k] = tv_k[2] + accv;
            }
        }
        lphi_k = h.lphi;
#pragma unroll
        for (int t = 0; t < 3; ++t) tv_k[t] = h.tv[t];
        gather_k = fast;
        q_k = c.q;
    }
}

// The persistent launch: the (tile, plane) pairs in tile-major order cut into
// equal contiguous ranges, one per workgroup (grid a multiple of 8).
__global__ void __launch_bounds__(kMThreads, 1) k_adj_antidiff_march(Geo g, MarchArgs a)
{
    __shared__ MarchLds S;
    const int nwg = gridDim.x;
    const int wg = fused::xcd_grouped_id();
    const long long total = (long long)a.tiles_x * a.tiles_y * g.nz;
    const long long span = (total + nwg - 1) / nwg;
    long long w0 = (long long)wg * span;
    const long long w1 = w0 + span < total ? w0 + span : total;
    while (w0 < w1) {
        const int tile = (int)(w0 / g.nz);
        const int kb = (int)(w0 - (long long)tile * g.nz);
        const int ke = (int)((long long)kb + (w1 - w0) < g.nz ? kb + (w1 - w0) : g.nz);
        w0 += ke - kb;
        march_segment(g, a, S, tile, kb, ke);
    }
}

#pragma clang fp contract(on)

}  // namespace adj
}  // namespace mpdata
