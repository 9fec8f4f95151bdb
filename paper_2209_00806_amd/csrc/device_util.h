// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "tbpm_internal.h"

namespace tbpm {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

template <typename R>
struct CxT;
template <>
struct CxT<double> {
    using T = d2;
};
template <>
struct CxT<float> {
    using T = f2;
};

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc += h * x for a real or complex matrix element h
template <typename C, typename R>
__device__ __forceinline__ C hmad(R h, C x, C acc) {
    acc.x = fma(h, x.x, acc.x);
    acc.y = fma(h, x.y, acc.y);
    return acc;
}
template <typename C>
__device__ __forceinline__ C hmad(C h, C x, C acc) {
    acc.x = fma(h.x, x.x, acc.x);
    acc.x = fma(-h.y, x.y, acc.x);
    acc.y = fma(h.x, x.y, acc.y);
    acc.y = fma(h.y, x.x, acc.y);
    return acc;
}

template <bool NT, typename T>
__device__ __forceinline__ T ldv(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stv(T *p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Blocks are dispatched round-robin over the 8 XCDs; remap so that XCD x
// works through one contiguous range of tiles (the neighbour rows gathered
// by a tile were then most likely brought into the same XCD's L2).  Launches
// that read what the previous launch wrote alternate the walking direction:
// the tiles a launch starts with are then the ones the previous launch
// finished with, whose rows are still in the caches.
// remap = g in 2..6: runs of G = 2^g consecutive tiles per XCD, the runs
// dealt to the XCDs in turn, so that a tile's neighbours in the row order
// share its XCD's L2 while all XCDs work on one compact front: block b (on
// XCD b & 7, its i = (b >> 3)-th there) takes tile ((i / G) 8 + (b & 7)) G +
// i mod G.  That maps every group of 8 G blocks onto the same 8 G tiles; the
// tiles past the last whole group are taken in order.
__device__ __forceinline__ int tile_of_block(int b, int n_tiles, int remap, int reverse = 0) {
    if (!remap) return reverse ? n_tiles - 1 - b : b;
    if (remap >= 2) {
        const int full = (n_tiles >> (remap + 3)) << (remap + 3);
        int t = b;
        if (b < full) {
            const int i = b >> 3;
            t = ((((i >> remap) << 3) + (b & 7)) << remap) + (i & ((1 << remap) - 1));
        }
        return reverse ? n_tiles - 1 - t : t;
    }
    const int q = n_tiles >> 3, r = n_tiles & 7;
    const int x = b & 7, i = b >> 3;
    // XCD x walks its contiguous range of q (+1) tiles, first to last or, with
    // reverse, last to first
    const int cnt = q + (x < r ? 1 : 0);
    return x * q + (x < r ? x : r) + (reverse ? cnt - 1 - i : i);
}

// Sum (dre, dim, nrm) over the threads of the workgroup that hold the same
// state (thread t holds state t & (S-1)) in a fixed order, and write the
// workgroup's partial sums for each state to out[(s*3 + q)*n_tiles + tile].
__device__ __forceinline__ void block_state_partials(double dre, double dim, double nrm, int log2s,
                                                     double *__restrict__ out, int tile, int n_tiles) {
    __shared__ double red[kWG / 64][64][3];
    const int S = 1 << log2s;
    for (int off = 32; off >= S; off >>= 1) {
        dre += __shfl_xor(dre, off);
        dim += __shfl_xor(dim, off);
        nrm += __shfl_xor(nrm, off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < S) {
        red[wave][lane][0] = dre;
        red[wave][lane][1] = dim;
        red[wave][lane][2] = nrm;
    }
    __syncthreads();
    if (threadIdx.x < S) {
        double a = 0, b = 0, c = 0;
#pragma unroll
        for (int w = 0; w < kWG / 64; ++w) {
            a += red[w][threadIdx.x][0];
            b += red[w][threadIdx.x][1];
            c += red[w][threadIdx.x][2];
        }
        const int64_t o = (int64_t)threadIdx.x * 3 * n_tiles + tile;
        out[o] = a;
        out[o + n_tiles] = b;
        out[o + 2 * (int64_t)n_tiles] = c;
    }
}

template <typename R, int VS>
using VecT = R __attribute__((ext_vector_type(2 * VS)));

template <typename R, bool CH>
struct HValT {
    using T = R;
};
template <typename R>
struct HValT<R, true> {
    using T = typename CxT<R>::T;
};

// acc_i += h * x_i for the VS complex components of a unit
template <typename R, int VS>
__device__ __forceinline__ void unit_mad_real(R h, VecT<R, VS> x, VecT<R, VS> &acc) {
#pragma unroll
    for (int i = 0; i < 2 * VS; ++i) acc[i] = fma(h, x[i], acc[i]);
}
template <typename R, int VS, typename C>
__device__ __forceinline__ void unit_mad_cplx(C h, VecT<R, VS> x, VecT<R, VS> &acc) {
#pragma unroll
    for (int i = 0; i < VS; ++i) {
        acc[2 * i] = fma(h.x, x[2 * i], acc[2 * i]);
        acc[2 * i] = fma(-h.y, x[2 * i + 1], acc[2 * i]);
        acc[2 * i + 1] = fma(h.x, x[2 * i + 1], acc[2 * i + 1]);
        acc[2 * i + 1] = fma(h.y, x[2 * i], acc[2 * i + 1]);
    }
}

// Per-state partial sums for units of VS states: lane l holds states
// (l & (U-1))*VS + i, U = units per row.  red: kWG/64 x 64 x 3 doubles of LDS
// that no thread of the workgroup uses any more.
template <int VS>
__device__ __forceinline__ void block_unit_partials(const double (&dre)[VS], const double (&dim)[VS],
                                                    const double (&nrm)[VS], int log2u,
                                                    double *__restrict__ out, int tile, int n_tiles,
                                                    double (*red)[64][3]) {
    const int U = 1 << log2u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < VS; ++i) {
        double a = dre[i], b = dim[i], c = nrm[i];
        for (int off = 32; off >= U; off >>= 1) {
            a += __shfl_xor(a, off);
            b += __shfl_xor(b, off);
            c += __shfl_xor(c, off);
        }
        if (lane < U) {
            red[wave][lane * VS + i][0] = a;
            red[wave][lane * VS + i][1] = b;
            red[wave][lane * VS + i][2] = c;
        }
    }
    __syncthreads();
    const int S = U * VS;
    if ((int)threadIdx.x < S) {
        double a = 0, b = 0, c = 0;
#pragma unroll
        for (int w = 0; w < kWG / 64; ++w) {
            a += red[w][threadIdx.x][0];
            b += red[w][threadIdx.x][1];
            c += red[w][threadIdx.x][2];
        }
        const int64_t o = (int64_t)threadIdx.x * 3 * n_tiles + tile;
        out[o] = a;
        out[o + n_tiles] = b;
        out[o + 2 * (int64_t)n_tiles] = c;
    }
}
template <int VS>
__device__ __forceinline__ void block_unit_partials(const double (&dre)[VS], const double (&dim)[VS],
                                                    const double (&nrm)[VS], int log2u,
                                                    double *__restrict__ out, int tile, int n_tiles) {
    __shared__ double red[kWG / 64][64][3];
    block_unit_partials<VS>(dre, dim, nrm, log2u, out, tile, n_tiles, red);
}

}  // namespace
}  // namespace tbpm
