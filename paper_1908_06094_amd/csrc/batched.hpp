// batched.hpp -- host driver of mpdata_run_batched: many independent
// problems, each with one or more tracers sharing its winds and metric, in
// one persistent launch per pass, all steps captured into a HIP graph.
//
// Work units of a pass are (problem, tile, tracer, plane); the units are cut
// into equal contiguous ranges per workgroup, so uneven problem sizes cost
// no load imbalance, and the tracers of one tile run on neighbouring
// workgroups of one XCD (their shared winds and G then come from that L2).
//
// The autotuner picks, per batch signature, the kernel variant: in FP32 the
// tile row width (16, 32 or 64 lanes: 12 x 44, 28 x 20 or 60 x 8 interior
// cells per 768-thread tile) and the workgroups per CU (one, or two with at
// most 80 registers); in both types whether the first corrective pass
// carries the donor-cell pass (as in the single-problem path) or a separate
// donor-cell kernel runs ahead of it.  It times one step of each on the
// caller's data; choices are kept in memory and appended to the file named
// by MPDATA_TUNE_CACHE.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mpdata.h"
#include "fused.hpp"
#include "donor.hpp"
#include "stages.hpp"

namespace batch {

using mpdata::Geo;
using mpdata::fused::BatchEntry;
using mpdata::fused::PassArgs;
using mpdata::stages::DonorEntry;

// Layout of the workspace: the entry tables first, then per item its
// per-tracer fields: X0, X1 (iterate ping-pong), S (step ping-pong) and, for
// three or more passes, two velocity triples.
struct Layout {
    size_t elem;
    int n, iters;
    std::vector<size_t> item_off;   // byte offset of item i's fields
    std::vector<long long> cells;
    std::vector<long long> vcells;  // elements of one tracer's velocity field (tile layout)
    size_t table_bytes;
    size_t total;
    int fields_per_tracer;
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline int tables_count(int iters) { return 2 + 2 * (iters - 1) + 1; }   // donor x2, passes x2, copy-back

inline Layout layout(const mpdata_problem* c, int n, const mpdata_batch_item* items)
{
    Layout L;
    L.elem = c->dtype == MPDATA_F64 ? 8 : 4;
    L.n = n;
    L.iters = c->iters;
    L.fields_per_tracer = 3 + (c->iters >= 3 ? 6 : 0);
    const size_t entry = std::max(sizeof(BatchEntry<double>),
                                  std::max(sizeof(DonorEntry<double>), sizeof(mpdata::fused::DonorBlocks<double>)));
    L.table_bytes = align256((size_t)tables_count(c->iters) * n * entry);
    size_t off = L.table_bytes;
    for (int i = 0; i < n; ++i) {
        const mpdata_batch_item& it = items[i];
        const long long cells = (long long)it.nx * it.ny * it.nz;
        const long long vcells = L.elem == 8 ? mpdata::fused::vel_elems<double>(it.nx, it.ny, it.nz)
                                             : mpdata::fused::vel_elems<float>(it.nx, it.ny, it.nz);
        L.cells.push_back(cells);
        L.vcells.push_back(vcells);
        L.item_off.push_back(off);
        off += align256((size_t)cells * it.ntracers * L.elem) * 3;
        if (L.fields_per_tracer > 3) off += align256((size_t)vcells * it.ntracers * L.elem) * 6;
    }
    L.total = off;
    return L;
}

template <class T>
struct ItemPtrs {
    T* user;           // the caller's psi (tracers consecutive)
    T* f[9];           // X0, X1, S, then velocity triples V0 (u, v, w), V1 (u, v, w)
};

template <class T>
ItemPtrs<T> item_ptrs(const Layout& L, char* ws, const mpdata_batch_item& it, int i)
{
    ItemPtrs<T> p;
    p.user = (T*)it.psi;
    const size_t fb = align256((size_t)L.cells[i] * it.ntracers * L.elem);
    const size_t vb = align256((size_t)L.vcells[i] * it.ntracers * L.elem);
    for (int f = 0; f < 9; ++f) {
        const size_t at = f < 3 ? fb * f : fb * 3 + vb * (f - 3);
        p.f[f] = f < L.fields_per_tracer ? (T*)(ws + L.item_off[i] + at) : nullptr;
    }
    return p;
}

inline Geo geo_of_item(const mpdata_problem* c, const mpdata_batch_item& it)
{
    Geo g;
    g.nx = it.nx;
    g.ny = it.ny;
    g.nz = it.nz;
    g.closed_x = c->bc[0] == MPDATA_CLOSED;
    g.closed_y = c->bc[1] == MPDATA_CLOSED;
    g.closed_z = c->bc[2] == MPDATA_CLOSED;
    g.sy = it.nx;
    g.sz = (long long)it.nx * it.ny;
    return g;
}

// Host copies of every table (uploaded once per call, ahead of the launches).
template <class T>
struct Tables {
    std::vector<mpdata::fused::DonorBlocks<T>> donor[2];  // by step parity
    std::vector<std::vector<BatchEntry<T>>> pass[2];    // [parity][m - 2]
    std::vector<DonorEntry<T>> copyback;                // S -> user (odd step counts)
    long long donor_total = 0, donor_blocks = 0;
    std::vector<long long> pass_total;                  // work units of pass m, [m - 2]
    bool fold = false;                                  // the first corrective pass runs the donor-cell pass
};

// Tables for the tile of row width LANES.  fold: the donor-cell pass runs
// inside the first corrective pass (its tile may be narrower, FP64).
template <class T, int LANES, int N = mpdata::fused::kThreads>
Tables<T> build_tables(const mpdata_problem* c, int n, const mpdata_batch_item* items, const Layout& L, char* ws,
                       bool fold)
{
    using TL = mpdata::fused::Tile<T, LANES, N>;
    Tables<T> tb;
    const int M = c->iters;
    const double eps = c->eps > 0.0 ? c->eps : 1e-15;
    tb.fold = fold && M >= 2;
    for (int par = 0; par < 2; ++par) tb.pass[par].resize(M > 1 ? M - 1 : 0);
    tb.pass_total.assign(M > 1 ? M - 1 : 0, 0);
    long long dbeg = 0, bbeg = 0;
    for (int i = 0; i < n; ++i) {
        const mpdata_batch_item& it = items[i];
        const ItemPtrs<T> P = item_ptrs<T>(L, ws, it, i);
        const Geo g = geo_of_item(c, it);
        const long long cells = L.cells[i];
        for (int par = 0; par < 2; ++par) {
            T* src = par == 0 ? P.user : P.f[2];
            T* dst = par == 0 ? P.f[2] : P.user;
            mpdata::fused::DonorBlocks<T> d;
            d.geo = g;
            d.phi = src;
            d.out = M == 1 ? dst : P.f[0];
            d.u = (const T*)it.cx;
            d.v = (const T*)it.cy;
            d.w = (const T*)it.cz;
            d.g = (const T*)it.g;
            d.stride = cells;
            d.block_begin = bbeg;
            d.bx = (it.nx + 63) / 64;
            d.by = (it.ny + 3) / 4;
            d.bz = (it.nz + mpdata::fused::kDonorChunk - 1) / mpdata::fused::kDonorChunk;
            d.tracers = it.ntracers;
            tb.donor[par].push_back(d);
            for (int m = 2; m <= M; ++m) {
                const bool donor = tb.fold && m == 2;
                const int tile_x = donor ? TL::donor_tile_x : TL::tile_x;
                const int tiles_x = (it.nx + tile_x - 1) / tile_x;
                const int tiles = tiles_x * ((it.ny + TL::tile_y - 1) / TL::tile_y);
                BatchEntry<T> e{};
                e.geo = g;
                PassArgs<T>& a = e.args;
                a.phi = donor ? nullptr : P.f[(m - 2) & 1];   // X_{m-1}: X0, X1, X0, ... (the donor-fused pass forms it)
                a.out = m == M ? dst : P.f[(m - 1) & 1];
                a.psin = src;
                if (m == 2) {
                    a.u = (const T*)it.cx;
                    a.v = (const T*)it.cy;
                    a.w = (const T*)it.cz;
                } else {
                    T* const* vin = &P.f[3 + 3 * ((m - 3) & 1)];
                    a.u = vin[0];
                    a.v = vin[1];
                    a.w = vin[2];
                }
                T* const* vout = &P.f[3 + 3 * ((m - 2) & 1)];
                a.ul = m < M ? vout[0] : nullptr;
                a.vl = m < M ? vout[1] : nullptr;
                a.wl = m < M ? vout[2] : nullptr;
                a.g = (const T*)it.g;
                a.eps = eps;
                a.tiles_x = tiles_x;
                a.tiles_y = (it.ny + TL::tile_y - 1) / TL::tile_y;
                e.begin = tb.pass_total[m - 2];
                e.tracer_stride = cells;
                e.vel_stride = L.vcells[i];
                e.tracers = it.ntracers;
                e.vel_per_tracer = m > 2;
                a.vel_tiled = m > 2 && TL::tiled_velocities;
                tb.pass[par][m - 2].push_back(e);
                if (par == 1) tb.pass_total[m - 2] += (long long)tiles * it.ntracers * it.nz;
            }
        }
        DonorEntry<T> cb;
        cb.geo = g;
        cb.phi = P.f[2];
        cb.out = P.user;
        cb.u = cb.v = cb.w = cb.g = nullptr;
        cb.begin = dbeg;
        cb.cells = cells;
        cb.stride = cells;
        cb.tracers = it.ntracers;
        tb.copyback.push_back(cb);
        const mpdata::fused::DonorBlocks<T>& d0 = tb.donor[0].back();
        bbeg += (long long)d0.bx * d0.by * d0.bz * it.ntracers;
        dbeg += cells * it.ntracers;
    }
    tb.donor_total = dbeg;
    tb.donor_blocks = bbeg;
    return tb;
}

template <class T>
__global__ void __launch_bounds__(256) k_copy_batched(const DonorEntry<T>* __restrict__ tab, int n_entries,
                                                      long long total)
{
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += step) {
        int lo = 0, hi = n_entries - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[mid].begin <= idx) lo = mid; else hi = mid - 1;
        }
        const DonorEntry<T>& e = tab[lo];
        const long long r = idx - e.begin;
        e.out[r] = e.phi[r];
    }
}

}  // namespace batch
