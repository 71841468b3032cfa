// common.hpp -- shared device helpers of the MPDATA HIP kernels (gfx950).
//
// Grid convention (paper, Section 3.1.4.1, the C-grid index convention):
// fields are dense [nz][ny][nx] arrays, i fastest; the face array of an axis
// shares the cell index space, slot i holding face i+1/2.  Periodic axes wrap
// (slot n-1 is the face n-1/2 == -1/2); closed axes carry no flux through the
// faces -1/2 and n-1/2 and clamp cell indices (a zero-gradient halo).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpdata {

struct Geo {
    int nx, ny, nz;
    int closed_x, closed_y, closed_z;
    long long sy, sz;   // strides of j and k in elements
};

// Neighbour cell index for i in [-1, n]: wraps on a periodic axis, clamps on
// a closed one.
__device__ __forceinline__ int nbr(int i, int n, int closed)
{
    if (i < 0) return closed ? 0 : n - 1;
    if (i >= n) return closed ? n - 1 : 0;
    return i;
}

// Value of face f+1/2 (f in [-1, n-1]) along an axis whose coordinate enters
// the linear index with `stride`, `base` being the index with that
// coordinate 0.  Closed walls (f == -1 or f == n-1) read as 0.
template <class T>
__device__ __forceinline__ T face_at(const T* __restrict__ a, long long base, long long stride,
                                     int f, int n, int closed)
{
    if (closed) {
        if (f < 0 || f >= n - 1) return T(0);
        return a[base + (long long)f * stride];
    }
    int ff = f < 0 ? n - 1 : f;
    return a[base + (long long)ff * stride];
}

template <class T> __device__ __forceinline__ T pos_part(T c) { return c > T(0) ? c : T(0); }
template <class T> __device__ __forceinline__ T neg_part(T c) { return c < T(0) ? c : T(0); }
template <class T> __device__ __forceinline__ T min2(T a, T b) { return a < b ? a : b; }
template <class T> __device__ __forceinline__ T max2(T a, T b) { return a > b ? a : b; }

template <class T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ a, long long n, T v)
{
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) a[q] = v;
}

}  // namespace mpdata
