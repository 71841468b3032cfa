// Donor-cell (upwind) pass kernels of the fast path: the first pass of every
// MPDATA step (Section 5; the edge and vertical fluxes and the divergence
// update of Listings 4-9), for one problem and for a batch of problems and
// tracers in one launch.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "fused.hpp"

namespace mpdata {
namespace fused {

// ---------------------------------------------------------------------------
// Donor-cell pass of the fast path: one thread per (i, j) column marching a
// chunk of levels; psi at k-1, k, k+1 and w at k-1/2 stay in registers, the
// x and y neighbours come through L1/L2.  HBM traffic: read psi, Cx, Cy, Cz,
// G and write psi^(1), once per cell.
// ---------------------------------------------------------------------------
constexpr int kDonorChunk = 16;

// Levels [k0, k1) of column (i, j).
template <class T>
__device__ __forceinline__ void donor_column(const Geo& g, const T* __restrict__ phi, const T* __restrict__ u,
                                             const T* __restrict__ v, const T* __restrict__ w,
                                             const T* __restrict__ gm, T* __restrict__ out, const int i, const int j,
                                             const int k0, const int k1)
{
    const long long col = (long long)j * g.sy + i;
    const long long c_im = (long long)j * g.sy + map_index(i - 1, g.nx, g.closed_x);
    const long long c_ip = (long long)j * g.sy + map_index(i + 1, g.nx, g.closed_x);
    const long long c_jm = (long long)map_index(j - 1, g.ny, g.closed_y) * g.sy + i;
    const long long c_jp = (long long)map_index(j + 1, g.ny, g.closed_y) * g.sy + i;
    // the face left of / below the cell: slot i-1 (wrapping) unless it is a wall
    const bool xr = !wall_face(i, g.nx, g.closed_x), xl = !wall_face(i - 1, g.nx, g.closed_x);
    const bool yr = !wall_face(j, g.ny, g.closed_y), yl = !wall_face(j - 1, g.ny, g.closed_y);
    const long long f_xl = (long long)j * g.sy + (i == 0 ? g.nx - 1 : i - 1);
    const long long f_yl = (long long)(j == 0 ? g.ny - 1 : j - 1) * g.sy + i;
    const T zero = T(0);

    auto plane = [&](int k) { return (long long)map_index(k, g.nz, g.closed_z) * g.sz; };
    auto wface = [&](int k) { return (w == nullptr || wall_face(k, g.nz, g.closed_z)) ? zero : w[plane(k) + col]; };
    T p_m = phi[plane(k0 - 1) + col];
    T p_c = phi[plane(k0) + col];
    T w_m = wface(k0 - 1);
    for (int k = k0; k < k1; ++k) {
        const long long b = (long long)k * g.sz;
        const T p_p = phi[plane(k + 1) + col];
        const T w_c = wface(k);
        const T ur = xr ? u[b + col] : zero, ul = xl ? u[b + f_xl] : zero;
        const T vr = yr ? v[b + col] : zero, vl = yl ? v[b + f_yl] : zero;
        const T fxr = pos_f(ur) * p_c + neg_f(ur) * phi[b + c_ip];
        const T fxl = pos_f(ul) * phi[b + c_im] + neg_f(ul) * p_c;
        const T fyr = pos_f(vr) * p_c + neg_f(vr) * phi[b + c_jp];
        const T fyl = pos_f(vl) * phi[b + c_jm] + neg_f(vl) * p_c;
        const T fzr = pos_f(w_c) * p_c + neg_f(w_c) * p_p;
        const T fzl = pos_f(w_m) * p_m + neg_f(w_m) * p_c;
        out[b + col] = p_c - (((fxr - fxl) + (fyr - fyl)) + (fzr - fzl)) / gm[b + col];
        p_m = p_c;
        p_c = p_p;
        w_m = w_c;
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_donor_march(Geo g, const T* __restrict__ phi, const T* __restrict__ u,
                                                     const T* __restrict__ v, const T* __restrict__ w,
                                                     const T* __restrict__ gm, T* __restrict__ out)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int k0 = blockIdx.z * kDonorChunk;
    const int k1 = k0 + kDonorChunk < g.nz ? k0 + kDonorChunk : g.nz;
    donor_column(g, phi, u, v, w, gm, out, i, j, k0, k1);
}

// The donor-cell pass over many problems and tracers: one block per
// (entry, tracer, 64x4 column tile, level chunk); entry e owns blocks
// [block_begin, block_begin + tracers * bx * by * bz).
template <class T>
struct DonorBlocks {
    Geo geo;
    const T* phi;      // tracer 0 (tracer t at + t * stride)
    T* out;
    const T* u;
    const T* v;
    const T* w;        // may be NULL
    const T* g;
    long long stride;
    long long block_begin;
    int bx, by, bz, tracers;
};

template <class T>
__global__ void __launch_bounds__(256) k_donor_march_batched(const DonorBlocks<T>* __restrict__ tab, int n_entries)
{
    const long long b = blockIdx.x;
    int lo = 0, hi = n_entries - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block_begin <= b) lo = mid; else hi = mid - 1;
    }
    const DonorBlocks<T>& e = tab[lo];
    const long long local = b - e.block_begin;
    const long long per_tracer = (long long)e.bx * e.by * e.bz;
    const int tracer = (int)(local / per_tracer);
    if (tracer >= e.tracers) return;
    int r = (int)(local - (long long)tracer * per_tracer);
    const int bz = r / (e.bx * e.by);
    r -= bz * e.bx * e.by;
    const int by = r / e.bx, bxi = r - by * e.bx;
    const int i = bxi * 64 + (int)(threadIdx.x & 63);
    const int j = by * 4 + (int)(threadIdx.x >> 6);
    if (i >= e.geo.nx || j >= e.geo.ny) return;
    const int k0 = bz * kDonorChunk;
    const int k1 = k0 + kDonorChunk < e.geo.nz ? k0 + kDonorChunk : e.geo.nz;
    const long long off = (long long)tracer * e.stride;
    donor_column(e.geo, e.phi + off, e.u, e.v, e.w, e.g, e.out + off, i, j, k0, k1);
}

}  // namespace fused
}  // namespace mpdata
