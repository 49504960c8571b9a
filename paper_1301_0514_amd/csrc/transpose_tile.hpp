// transpose_tile.hpp -- one unit of an out-of-place N x N transpose through
// LDS: 64 source rows by 128 source columns (two 64 x 64 tiles side by side).
// Used by the standalone batched transpose and by row passes that carry a
// transpose as extra workgroups of their own launch.
//
// The tiles are held as element pairs (16 bytes for complex64, 8 for float):
// a lane loads one pair of a source row, so each source row is read as one
// contiguous 1 KB (512 B) run.  On the way out a lane takes the pair of
// columns (2q, 2q+1) from the two source rows (2l, 2l+1), transposes that
// 2 x 2 block in registers and writes one pair to each of the output rows 2q
// and 2q+1, as contiguous runs.  Pair q of tile row y is kept in LDS slot
// q ^ ((y >> 1) & 31): the 32 lanes that read one pair column then touch 32
// distinct slots, and each row's write is a permutation within the row, so
// neither phase has bank conflicts.  N is even (every supported size is), so
// a pair never straddles the edge of a ragged tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scint {

template <typename T> struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};

constexpr int kTransposeTilesX = 2;
constexpr int kTransposeUnitCols = 64 * kTransposeTilesX;  // source columns per unit
constexpr int kTransposeUnitRows = 64;                     // source rows per unit

template <typename T> struct TransposeTile {
    Pair<T> p[kTransposeTilesX][64][32];
};

// Loads and stores of one pair, plain or nontemporal (streamed past the
// caches' reuse, so that a transpose running beside other work does not evict
// that work's cached data)
template <typename T, bool NTMP> __device__ __forceinline__ Pair<T> pair_load(const T *p) {
    if constexpr (NTMP) {
        using V = float __attribute__((ext_vector_type(sizeof(Pair<T>) / 4)));
        const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
        return __builtin_bit_cast(Pair<T>, v);
    } else {
        return *reinterpret_cast<const Pair<T> *>(p);
    }
}
template <typename T, bool NTMP> __device__ __forceinline__ void pair_store(T *p, const Pair<T> &x) {
    if constexpr (NTMP) {
        using V = float __attribute__((ext_vector_type(sizeof(Pair<T>) / 4)));
        __builtin_nontemporal_store(__builtin_bit_cast(V, x), reinterpret_cast<V *>(p));
    } else {
        *reinterpret_cast<Pair<T> *>(p) = x;
    }
}

__host__ __device__ inline int transpose_units_x(int N) { return (N + kTransposeUnitCols - 1) / kTransposeUnitCols; }
__host__ __device__ inline int transpose_units_y(int N) { return (N + kTransposeUnitRows - 1) / kTransposeUnitRows; }

// Transposes unit (ux, uy) of src into dst (both N x N, row-major), with NT
// threads of the workgroup (NT >= 128: the 256 lane roles are spread over
// them; threads beyond 256 only take part in the barrier); NTMP selects
// nontemporal global accesses.  One barrier separates the LDS writes from
// the reads; the caller places another before the tile is reused.
template <typename T, int NT, bool NTMP = false>
__device__ __forceinline__ void transpose_unit(const T *__restrict__ src, T *__restrict__ dst, int N, int ux, int uy,
                                               TransposeTile<T> &tile, int tid) {
    static_assert(NT >= 128, "the transpose unit needs at least 128 threads");
    constexpr int VT = (256 + NT - 1) / NT;  // lane roles per thread
    const int y0 = uy * 64;
    // Unguarded loads at addresses clamped into the matrix, so that all of
    // them are in flight at once (a guarded load is waited for on its own).
    // The slots they fill for positions outside the matrix are never read.
    Pair<T> v[VT][kTransposeTilesX][8];
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int role = tid + k * NT;
        if (VT > 1 && role >= 256) break;
        const int lx = role % 32, ly = role / 32;
#pragma unroll
        for (int tt = 0; tt < kTransposeTilesX; ++tt) {
            const int xc = min((ux * kTransposeTilesX + tt) * 64 + 2 * lx, N - 2);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int yc = min(y0 + ly + 8 * i, N - 1);
                v[k][tt][i] = pair_load<T, NTMP>(src + (int64_t)yc * N + xc);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int role = tid + k * NT;
        if (role < 256) {
            const int lx = role % 32, ly = role / 32;
#pragma unroll
            for (int tt = 0; tt < kTransposeTilesX; ++tt) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = ly + 8 * i;
                    tile.p[tt][r][lx ^ ((r >> 1) & 31)] = v[k][tt][i];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VT; ++k) {
        const int role = tid + k * NT;
        if (role < 256) {
            const int lx = role % 32, ly = role / 32;
            const int ya = y0 + 2 * lx;
#pragma unroll
            for (int tt = 0; tt < kTransposeTilesX; ++tt) {
                const int x0 = (ux * kTransposeTilesX + tt) * 64;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = ly + 8 * i, x = x0 + 2 * q;  // output rows x, x + 1
                    if (x < N && ya < N) {
                        const Pair<T> u = tile.p[tt][2 * lx][q ^ lx];      // source row ya: columns x, x + 1
                        const Pair<T> w = tile.p[tt][2 * lx + 1][q ^ lx];  // source row ya + 1
                        pair_store<T, NTMP>(dst + (int64_t)x * N + ya, Pair<T>{u.a, w.a});
                        pair_store<T, NTMP>(dst + (int64_t)(x + 1) * N + ya, Pair<T>{u.b, w.b});
                    }
                }
            }
        }
    }
}

}  // namespace scint
