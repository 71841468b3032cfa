// unstructured.hpp -- the edge-based donor-cell (upwind) step of the paper's
// own MPDATA dwarf on an unstructured mesh (Section 5, Listings 4-9): upwind
// flux on every edge, vertical upwind flux with the boundary factor pivbz
// (Listing 7), flux divergence at the nodes over the dual volume (Listing 8)
// and the solution update, fused into one kernel (the fusion of Listing 9
// and Table 2: no edge flux or vertical flux reaches memory).
//
// Mapping onto gfx950: fields are (node, level) with the level fastest; a
// wave takes one node and its lanes run over the levels, so the node's
// connectivity is read once per wave through scalar loads and every gather
// through it (psi at an edge's end nodes, the edge's vn) is a contiguous run
// of levels: coalesced whatever the node numbering.  (The paper reaches
// coalescing on the GPU through a structured, coloured numbering of the
// mesh, Figures 9-12 and Table 1; with levels innermost the numbering only
// affects cache reuse.)  Each wave gathers over its node's edges in the
// node-to-edge table's order and recomputes the edge fluxes it needs (each
// edge flux is formed by both of its end nodes), so there are no atomics
// and the result is deterministic.
//
// Arithmetic: no contraction, the order of the stages' formulas; the
// results equal the per-stage evaluation bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpdata {
namespace unstructured {

#pragma clang fp contract(off)

template <class T>
struct UArgs {
    const int32_t* edge_nodes;   // (edges, 2): ip1, ip2
    const int32_t* node_ptr;     // (nodes + 1)
    const int32_t* node_edges;   // (node_ptr[nodes])
    const int8_t* node_sign;     // +1: the node is the edge's ip1, -1: its ip2
    const T* vol;                // (nodes) dual volumes
    const T* psi;                // (nodes, nz)
    const T* vn;                 // (edges, nz)
    const T* w;                  // (nodes, nz), w[n][k] at the interface k-1 / k; NULL: no vertical wind
    const T* rho;                // (nodes, nz)
    T* out;                      // (nodes, nz)
    T pivbz;
    int32_t n_nodes, nz;
};

constexpr int kGroup = 8;   // edges whose loads are in flight together

template <class T> __device__ __forceinline__ T upos(T c) { return c > T(0) ? c : T(0); }
template <class T> __device__ __forceinline__ T uneg(T c) { return c < T(0) ? c : T(0); }

// One wave per node: the node's connectivity is wave-uniform (scalar loads),
// the lanes run over the levels in chunks of 64.  The dispatcher deals
// workgroups round-robin over the 8 XCDs; the logical id gives each XCD a
// contiguous range of nodes, so neighbouring nodes (which read each other's
// psi and share their edges' vn) meet in one L2.  gridDim.x is a multiple of 8.
template <class T>
__device__ __forceinline__ T ustep_point(const UArgs<T>& a, long long c, int k, T acc, T rvol)
{
    // vertical: interface fluxes below (k) and above (k+1) the level (Listing 7)
    T fzb = T(0), fzt = T(0);
    if (a.w != nullptr && a.nz > 1) {
        auto fint = [&](int kk) {
            const T wv = a.w[c + kk];
            return upos(wv) * a.psi[c + kk - 1] + uneg(wv) * a.psi[c + kk];
        };
        fzb = k == 0 ? a.pivbz * fint(1) : fint(k);
        fzt = k == a.nz - 1 ? a.pivbz * fint(a.nz - 1) : fint(k + 1);
    }
    const T div = acc / rvol + (fzt - fzb);
    return a.psi[c + k] - div / a.rho[c + k];
}

// One wave per node (the former mapping, kept for comparison): the node's
// connectivity is wave-uniform (scalar loads), the lanes run over the levels
// in chunks of 64.
template <class T>
__global__ void __launch_bounds__(256) k_ustep_wave(UArgs<T> a)
{
    const int wg = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int n = __builtin_amdgcn_readfirstlane(wg * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (n >= a.n_nodes) return;
    const int lane = threadIdx.x & 63;
    const long long nz = a.nz;
    const long long c = (long long)n * nz;
    const int j0 = a.node_ptr[n], j1 = a.node_ptr[n + 1];
    const T rvol = a.vol[n];
    // two 64-level chunks per pass (levels k and k + 64), so that twice as
    // many loads are in flight per wave
    for (int k0 = 0; k0 < a.nz; k0 += 128) {
        const int k = k0 + lane, k2 = k + 64;
        if (k >= a.nz) break;
        const bool two = k2 < a.nz;
        const int kk2 = two ? k2 : k;   // a valid level for the second chunk's loads
        T acc = T(0), acc2 = T(0);
        for (int jb = j0; jb < j1; jb += kGroup) {
            T f[kGroup], f2[kGroup], sg[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                f[q] = f2[q] = sg[q] = T(0);
                const int j = jb + q;
                if (j < j1) {
                    const long long e = a.node_edges[j];
                    const long long ip1 = a.edge_nodes[2 * e], ip2 = a.edge_nodes[2 * e + 1];
                    const T v = a.vn[e * nz + k], v2 = a.vn[e * nz + kk2];
                    f[q] = upos(v) * a.psi[ip1 * nz + k] + uneg(v) * a.psi[ip2 * nz + k];
                    f2[q] = upos(v2) * a.psi[ip1 * nz + kk2] + uneg(v2) * a.psi[ip2 * nz + kk2];
                    sg[q] = (T)a.node_sign[j];
                }
            }
#pragma unroll
            for (int q = 0; q < kGroup; ++q)
                if (jb + q < j1) {
                    acc += sg[q] * f[q];
                    acc2 += sg[q] * f2[q];
                }
        }
        a.out[c + k] = ustep_point(a, c, k, acc, rvol);
        if (two) a.out[c + k2] = ustep_point(a, c, k2, acc2, rvol);
    }
}

// Four nodes per wave: each node takes a group of kLevelLanes lanes, which
// run over its levels in blocks of kLevelLanes (one 128-byte line of FP64
// per gather).  Every lane of the wave works on every level block (a column
// of 80 levels fills 5 blocks exactly) and the four nodes' gathers are in
// flight together.  A node's connectivity (up to kGroup edges: the edge's
// and its two end nodes' element offsets and the sign) is read once, by
// vector loads its group's lanes share, and kept in registers across the
// level blocks; the offsets are 32-bit (the host uses the one-wave kernel
// for meshes whose (node or edge) x level count reaches 2^31).  Edges are
// summed in the node-to-edge table's order, as in the one-wave mapping.
// Lanes per node (a build option; on O128 x 80 levels 16 measured 145 us,
// 32 lanes 180 us, 8 lanes 170 us).
#ifndef MPDATA_USTEP_LANES
#define MPDATA_USTEP_LANES 16
#endif
constexpr int kLevelLanes = MPDATA_USTEP_LANES;
constexpr int kNodesPerWave = 64 / kLevelLanes;

template <class T>
__global__ void __launch_bounds__(256) k_ustep(UArgs<T> a)
{
    const int wg = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int lane = threadIdx.x & 63;
    const int sub = lane & (kLevelLanes - 1);
    const int n = (wg * (blockDim.x >> 6) + (int)(threadIdx.x >> 6)) * kNodesPerWave + lane / kLevelLanes;
    const bool node_ok = n < a.n_nodes;
    const int nn = node_ok ? n : a.n_nodes - 1;   // every load stays in range
    const int nz = a.nz;
    const int c = nn * nz;
    const int j0 = a.node_ptr[nn], j1 = a.node_ptr[nn + 1];
    const T rvol = a.vol[nn];
    int eo[kGroup], p1[kGroup], p2[kGroup];
    T sg[kGroup];
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
        const int j = j0 + q < j1 ? j0 + q : j0;   // a valid entry (degree >= 1 where used)
        const int e = j0 < j1 ? a.node_edges[j] : 0;
        eo[q] = e * nz;
        p1[q] = (j0 < j1 ? a.edge_nodes[2 * e] : nn) * nz;
        p2[q] = (j0 < j1 ? a.edge_nodes[2 * e + 1] : nn) * nz;
        sg[q] = j0 + q < j1 ? (T)a.node_sign[j] : T(0);
    }
    for (int k0 = 0; k0 < nz; k0 += kLevelLanes) {
        const int k = k0 + sub;
        const bool ok = node_ok && k < nz;
        const int kk = k < nz ? k : nz - 1;
        T f[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            f[q] = T(0);
            if (j0 + q < j1) {
                const T v = a.vn[eo[q] + kk];
                f[q] = upos(v) * a.psi[p1[q] + kk] + uneg(v) * a.psi[p2[q] + kk];
            }
        }
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < kGroup; ++q)
            if (j0 + q < j1) acc += sg[q] * f[q];
        // nodes of a higher degree than kGroup (none on the octahedral grid)
        for (int j = j0 + kGroup; j < j1; ++j) {
            const long long e = a.node_edges[j];
            const long long ip1 = a.edge_nodes[2 * e], ip2 = a.edge_nodes[2 * e + 1];
            const T v = a.vn[e * nz + kk];
            acc += (T)a.node_sign[j] * (upos(v) * a.psi[ip1 * nz + kk] + uneg(v) * a.psi[ip2 * nz + kk]);
        }
        const T r = ustep_point(a, (long long)c, kk, acc, rvol);
        if (ok) a.out[c + k] = r;
    }
}

#pragma clang fp contract(on)

}  // namespace unstructured
}  // namespace mpdata
