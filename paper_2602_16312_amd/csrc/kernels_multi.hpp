// Multi-right-hand-side variants of the per-step kernels: R independent
// columns share every operator, transfer and smoother load.  Vectors are
// RHS-minor: entry (DoF t, column r) at t*R + r.  Included by solver.hip
// after kernels.hpp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dgmg {

typedef float v4f __attribute__((ext_vector_type(4)));

// Orders one wave's LDS accesses at the compiler level.  Only lanes of one
// wave exchange data through the buffers it guards, and LDS executes a
// wave's instructions in issue order, so no barrier is needed.
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc[r] += (A (va + vb))[row, r] for the tile thread (lc, i), slot by slot:
// one coalesced block column value per (slot, j) and the R contiguous
// gathered values of the column cell.
// Neighbour segments (B rows of R values) for cells whose B lanes share a
// wave are staged in a wave-private LDS buffer: lane i loads row i and every
// lane reads the B rows back (one address per cell: LDS broadcast), instead
// of every lane loading the whole segment through the address unit.  The
// cell buffers are padded by 16 bytes against bank conflicts.
template <int B>
constexpr bool stage_segments() { return 64 % B == 0; }
template <typename T, int B, int R>
__device__ __forceinline__ T* segment_buffer() {
    constexpr int CS = B * R + 16 / (int)sizeof(T);
    __shared__ __align__(16) T stage[stage_segments<B>() ? kWG / 64 * (64 / B) * CS : 1];
    if constexpr (!stage_segments<B>()) return stage;
    return stage + ((threadIdx.x >> 6) * (64 / B) + ((threadIdx.x & 63) / B)) * CS;
}
// acc[r] += sum_j a[j] (va + vb)[nb, j, r] at row i of the thread's cell
// (cs: the cell's buffer from segment_buffer).
template <typename T, int B, int R, bool VB>
__device__ __forceinline__ void segment_accumulate(const T* __restrict__ va, const T* __restrict__ vb,
                                                   int nb, int i, const T* a, T* acc, T* cs) {
    auto column = [&](int j, int r) -> T {
        const size_t k = ((size_t)nb * B + j) * R + r;
        return VB ? va[k] + vb[k] : va[k];
    };
    if constexpr (stage_segments<B>()) {
        T row[R];
#pragma unroll
        for (int r = 0; r < R; ++r) row[r] = column(i, r);
        wave_lds_fence();   // the previous segment's reads stay before these writes
#pragma unroll
        for (int r = 0; r < R; ++r) cs[i * R + r] = row[r];
        wave_lds_fence();
#pragma unroll
        for (int j = 0; j < B; ++j)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += a[j] * cs[j * R + r];
    } else {
#pragma unroll
        for (int j = 0; j < B; ++j)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += a[j] * column(j, r);
    }
}

template <typename T, int B, int R, bool VB>
__device__ __forceinline__ void ell_row_apply_m(const LevelArgs<T>& L, int tile, int lc,
                                                const T* __restrict__ va, const T* __restrict__ vb,
                                                T* acc) {
    constexpr int TC = Tile<T, B>::TC, TR = Tile<T, B>::TR;
    const int i = threadIdx.x - lc * B;
    const int s0 = L.slot_ptr[tile], ns = L.slot_ptr[tile + 1] - s0;
    const T* __restrict__ A = L.vals + (size_t)s0 * B * TR + threadIdx.x;
    const int32_t* __restrict__ nbp = L.snb + (size_t)s0 * TC + lc;
    T* cs = segment_buffer<T, B, R>();
    for (int s = 0; s < ns; ++s) {
        const int nb = nbp[(size_t)s * TC];
        T a[B];
#pragma unroll
        for (int j = 0; j < B; ++j) a[j] = A[((size_t)s * B + j) * TR];
        segment_accumulate<T, B, R, VB>(va, vb, nb, i, a, acc, cs);
    }
}

// Axis-ELL variant: the upper face slots, the cell block from its symmetric
// planes (plane k: A[i][i+k] and, at row i-k, A[i][i-k]), then the lower
// faces read transposed.
template <typename T, int B, int R, bool VB>
__device__ __forceinline__ void ax_row_apply_m(const LevelArgs<T>& L, int tile, int lc, int cell,
                                               const T* __restrict__ va, const T* __restrict__ vb,
                                               T* acc) {
    constexpr int TC = Tile<T, B>::TC, TR = Tile<T, B>::TR, D = dim_of<B>();
    constexpr int P0 = ax_cell_planes(B), TP = ax_tile_planes(B, D);
    const int i = threadIdx.x - lc * B;
    const T* __restrict__ A = L.vals + (size_t)tile * TP * TR + threadIdx.x;
    auto column = [&](int nb, int j, int r) -> T {
        const size_t k = ((size_t)nb * B + j) * R + r;
        return VB ? va[k] + vb[k] : va[k];
    };
    T* cs = segment_buffer<T, B, R>();
    auto accumulate = [&](const T* a, int nb) { segment_accumulate<T, B, R, VB>(va, vb, nb, i, a, acc, cs); };
    for (int s = 0; s < D; ++s) {
        const int nb = L.up[(size_t)s * L.n + cell];
        T a[B];
#pragma unroll
        for (int j = 0; j < B; ++j) a[j] = A[(size_t)(P0 + s * B + j) * TR];
        accumulate(a, nb);
    }
    if constexpr (stage_segments<B>()) {
        // the cell's B lanes sit in one wave: each loads its own row of the
        // segment, rows i + k arrive by lane shuffles, and so do the products
        // A[i-k][i] x[i-k][r] of row i - k (the symmetric entries)
        const int base = ((int)threadIdx.x & 63) - i;
        T xs[R];
#pragma unroll
        for (int r = 0; r < R; ++r) xs[r] = column(cell, i, r);
#pragma unroll
        for (int k = 0; k < P0; ++k) {
            const T ao = A[(size_t)k * TR];
            if (k == 0) {
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += ao * xs[r];
                continue;
            }
            const int jp = i + k >= B ? i + k - B : i + k;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += ao * __shfl(xs[r], base + jp, 64);
            if (2 * k != B) {
                const int jm = i >= k ? i - k : i - k + B;
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += __shfl(ao * xs[r], base + jm, 64);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < P0; ++k) {
            const int jp = i + k >= B ? i + k - B : i + k;
            const T ao = A[(size_t)k * TR];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += ao * column(cell, jp, r);
            if (k > 0 && 2 * k != B) {
                const int jm = i >= k ? i - k : i - k + B;
                const T am = A[(ptrdiff_t)k * TR + (jm - i)];
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += am * column(cell, jm, r);
            }
        }
    }
    for (int ax = 0; ax < D; ++ax) {
        const int c0 = L.lo[(size_t)ax * L.n + cell];
        if (c0 < 0) continue;
        const int t0 = c0 / TC, l0 = c0 - t0 * TC;
        const T* At = L.vals + ((size_t)t0 * TP + P0 + ax * B + i) * TR + (size_t)l0 * B;
        T a[B];
#pragma unroll
        for (int r = 0; r < B; ++r) a[r] = At[r];
        accumulate(a, c0);
    }
}

template <typename T, int B, int R, bool VB, bool AX>
__device__ __forceinline__ void row_apply_m(const LevelArgs<T>& L, int tile, int lc, int cell,
                                            const T* __restrict__ va, const T* __restrict__ vb, T* acc) {
    if constexpr (AX)
        ax_row_apply_m<T, B, R, VB>(L, tile, lc, cell, va, vb, acc);
    else
        ell_row_apply_m<T, B, R, VB>(L, tile, lc, va, vb, acc);
}

template <bool AX, bool VB>
__device__ __forceinline__ void mfma8_tile_product(const LevelArgs<float>& L, int tile,
                                                   const float* __restrict__ va,
                                                   const float* __restrict__ vb, float* acc);

// Workgroup sums of R doubles into partial[blockIdx.x * R + r].
template <int R>
__device__ __forceinline__ void wg_sum_store_m(const double* v, double* partial) {
    __shared__ double red[kWG / 64][R];
    double w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        w[r] = v[r];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w[r] += __shfl_xor(w[r], off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int r = 0; r < R; ++r) red[wv][r] = w[r];
    __syncthreads();
    if ((int)threadIdx.x < R) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k][threadIdx.x];
        partial[(size_t)blockIdx.x * R + threadIdx.x] = s;
    }
}

// y = A va; optional per-column partial of dot(w, y).
template <typename T, int B, int R, bool AX>
__global__ __launch_bounds__(kWG) void k_apply_m(LevelArgs<T> L, const T* __restrict__ va,
                                                 T* __restrict__ y, const T* __restrict__ w,
                                                 double* __restrict__ partial) {
    DGMG_TILE_THREAD(T, B)
    double contrib[R];
#pragma unroll
    for (int r = 0; r < R; ++r) contrib[r] = 0.0;
    if (active) {
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0;
        row_apply_m<T, B, R, false, AX>(L, tile, lc, cell, va, nullptr, acc);
        T* yp = y + (size_t)t * R;
#pragma unroll
        for (int r = 0; r < R; ++r) yp[r] = acc[r];
        if (w) {
            const T* wp = w + (size_t)t * R;
            T wv[R];
#pragma unroll
            for (int r = 0; r < R; ++r) wv[r] = wp[r];
#pragma unroll
            for (int r = 0; r < R; ++r) contrib[r] = (double)wv[r] * (double)acc[r];
        }
    }
    if (partial) wg_sum_store_m<R>(contrib, partial);
}

// Residual per column r = rhs - A (va + vb) with the same optional epilogues
// as the single-column kernel (d, xout, per-column ||r||^2, restriction
// partials).
template <typename T, int B, int R, bool VB, bool AX, bool MF = false>
__global__ __launch_bounds__(kWG) void k_residual_m(LevelArgs<T> L, const T* __restrict__ va,
                                                    const T* __restrict__ vb, const T* __restrict__ rhs,
                                                    T* __restrict__ r, T* __restrict__ d, T c1,
                                                    T* __restrict__ xout, double* __restrict__ partial,
                                                    const T* __restrict__ P, T* __restrict__ rp,
                                                    const int32_t* __restrict__ ptype) {
    DGMG_TILE_THREAD(T, B)
    double contrib[R];
    T rr[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        contrib[q] = 0.0;
        rr[q] = 0;
    }
    T acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0;
    if constexpr (MF) mfma8_tile_product<AX, VB>(L, tile, va, vb, acc);   // whole workgroup
    if (active) {
        // own rows first (all loads of a kind issued together), then the product
        const size_t k0 = (size_t)t * R;
        T bv[R], xs[R];
#pragma unroll
        for (int q = 0; q < R; ++q) bv[q] = rhs[k0 + q];
        if (xout) {
#pragma unroll
            for (int q = 0; q < R; ++q) xs[q] = VB ? va[k0 + q] + vb[k0 + q] : va[k0 + q];
        }
        if constexpr (!MF) row_apply_m<T, B, R, VB, AX>(L, tile, lc, cell, va, vb, acc);
        const T di = L.dinv[t];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            rr[q] = bv[q] - acc[q];
            contrib[q] = (double)rr[q] * (double)rr[q];
        }
        if (r) {
#pragma unroll
            for (int q = 0; q < R; ++q) r[k0 + q] = rr[q];
        }
        if (d) {
#pragma unroll
            for (int q = 0; q < R; ++q) d[k0 + q] = di * rr[q] * c1;
        }
        if (xout) {
#pragma unroll
            for (int q = 0; q < R; ++q) xout[k0 + q] = xs[q];
        }
    }
    if (P) {
        __shared__ T rs[kWG * R];
#pragma unroll
        for (int q = 0; q < R; ++q) rs[threadIdx.x * R + q] = rr[q];
        __syncthreads();
        if (active) {
            constexpr int TR = Tile<T, B>::TR;
            const int j = threadIdx.x - lc * B;
            const T* Pc = ptype ? P + (size_t)ptype[cell] * B * B + j : P + ((size_t)tile * B + j) * TR + lc * B;
            const int ks = ptype ? B : 1;
            T s[R];
#pragma unroll
            for (int q = 0; q < R; ++q) s[q] = 0;
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const T pk = Pc[k * ks];
#pragma unroll
                for (int q = 0; q < R; ++q) s[q] += pk * rs[(lc * B + k) * R + q];
            }
#pragma unroll
            for (int q = 0; q < R; ++q) rp[(size_t)t * R + q] = s[q];
        }
    }
    if (partial) wg_sum_store_m<R>(contrib, partial);
}

// Epilogue of the Chebyshev step for one row t and its R columns: x += d
// (x = d when assign), r -= A d, dn = cd d + cr dinv r.  Each array's R
// contiguous entries are loaded together (vector loads) before any store.
template <typename T, int R>
__device__ __forceinline__ void cheb_epilogue_m(const LevelArgs<T>& L, int t, const T* acc,
                                                const T* __restrict__ d, T* __restrict__ x,
                                                T* __restrict__ r, T* __restrict__ dn, T cd, T cr,
                                                int assign, int last) {
    const size_t k0 = (size_t)t * R;
    T dv[R], rv[R], xv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) dv[q] = d[k0 + q];
#pragma unroll
    for (int q = 0; q < R; ++q) rv[q] = r[k0 + q];
    if (!assign) {
#pragma unroll
        for (int q = 0; q < R; ++q) xv[q] = x[k0 + q];
    } else {
#pragma unroll
        for (int q = 0; q < R; ++q) xv[q] = 0;
    }
    const T di = L.dinv[t];
    if (last) {
        // the sweep's final correction applied at once (as the single-column step)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const T rr = rv[q] - acc[q];
            const T dnew = cd * dv[q] + cr * di * rr;
            x[k0 + q] = (xv[q] + dv[q]) + dnew;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const T rr = rv[q] - acc[q];
        x[k0 + q] = xv[q] + dv[q];
        r[k0 + q] = rr;
        dn[k0 + q] = cd * dv[q] + cr * di * rr;
    }
}

// One inner Chebyshev step on R columns (VALU).
template <typename T, int B, int R, bool AX>
__global__ __launch_bounds__(kWG) void k_cheb_step_m(LevelArgs<T> L, const T* __restrict__ d,
                                                     T* __restrict__ x, T* __restrict__ r,
                                                     T* __restrict__ dn, T cd, T cr, int assign,
                                                     int last) {
    DGMG_TILE_THREAD(T, B)
    if (!active) return;
    T acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0;
    row_apply_m<T, B, R, false, AX>(L, tile, lc, cell, d, nullptr, acc);
    cheb_epilogue_m<T, R>(L, t, acc, d, x, r, dn, cd, cr, assign, last);
}

// A (va + vb) for a whole tile of FP32 8x8 blocks and 8 columns on the
// matrix cores; every thread of the workgroup must call it.  Per wave 8
// cells x 8 rows; v_mfma_f32_4x4x1f32 (16 blocks of 4x4) with block =
// (cell, half of the rows) takes the stored value of the lane's (cell, row)
// as its A operand (lane 4*blk + i supplies row i) and the gathered column
// values as B (lane 4*blk + j supplies column j of one half of the
// right-hand sides); lane 4*blk + j then holds rows 4*half + 0..3 of
// right-hand side 4*rh + j, which LDS hands to the thread of each row
// (acc[0..7] = the row's 8 columns).  On the axis-ELL layout the lower faces
// contribute the transposed stored block (A operand = column of the
// neighbour's block, zero where the cell has no lower neighbour).
//
// The B operands of a lane are 16 values at a stride of 4 floats inside the
// neighbour's 8x8 segment (256 contiguous bytes).  Gathering them directly
// costs 16 vector-memory instructions per neighbour, each touching 8 cache
// lines, which saturates the texture-address unit.  Instead the 8 lanes of
// a cell read the segment with two 16-byte loads each into a wave-private
// LDS buffer and every lane reads its 16 operands back from there (8
// two-address LDS reads).  Only lanes of one wave exchange data through the
// buffer, and LDS executes a wave's instructions in issue order, so a
// wave-level compiler fence is all the ordering needed.

template <bool AX, bool VB>
__device__ __forceinline__ void mfma8_tile_product(const LevelArgs<float>& L, int tile,
                                                   const float* __restrict__ va,
                                                   const float* __restrict__ vb, float* acc) {
    constexpr int B = 8, R = 8, TC = Tile<float, 8>::TC, TR = Tile<float, 8>::TR;
    // cell stride in the staging buffer: 64 floats + 4 of padding, so that
    // the 8 cells' reads at one offset land in distinct banks
    constexpr int XS = 68;
    __shared__ __align__(16) float xstage[(kWG / 64) * 8 * XS];
    const int lane = threadIdx.x & 63;
    const int lc = threadIdx.x / B;
    const int row = threadIdx.x - lc * B;
    const int cell0 = tile * TC;
    const int mycell = min(cell0 + lc, L.n - 1);    // padding lanes reuse a valid cell
    const int jj = lane & 3;                        // B operand / result column in block
    const int g = lane >> 3, q8 = lane & 7;         // the lane's cell in the wave, its 16-byte chunk
    float* xw = xstage + (threadIdx.x >> 6) * 8 * XS + g * XS;
    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    // the lane's two 16-byte chunks of the neighbour segment (va + vb)
    auto load_seg = [&](int nb, v4f& u0, v4f& u1) {
        const v4f* xv = reinterpret_cast<const v4f*>(va + (size_t)nb * B * R) + q8;
        u0 = xv[0];
        u1 = xv[8];
        if constexpr (VB) {
            const v4f* yv = reinterpret_cast<const v4f*>(vb + (size_t)nb * B * R) + q8;
            u0 += yv[0];
            u1 += yv[8];
        }
    };
    auto mma_seg = [&](const float* a, const v4f& u0, const v4f& u1) {
        wave_lds_fence();   // the previous neighbour's reads stay before these writes
        *reinterpret_cast<v4f*>(xw + 4 * q8) = u0;
        *reinterpret_cast<v4f*>(xw + 32 + 4 * q8) = u1;
        wave_lds_fence();
        float b0[B], b1[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            b0[j] = xw[j * R + jj];
            b1[j] = xw[j * R + 4 + jj];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            acc0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[j], b0[j], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a[j], b1[j], acc1, 0, 0, 0);
        }
    };
    auto mma = [&](const float* a, int nb) {
        v4f u0, u1;
        load_seg(nb, u0, u1);
        mma_seg(a, u0, u1);
    };
    if constexpr (AX) {
        // 7 neighbours: self and the three upper faces (stored blocks), the
        // three lower faces (transposed blocks of the lower neighbour).
        // Without vb all 7 segments are requested at the start: a wave then
        // touches each cache line within one memory round trip instead of
        // over its whole lifetime, so the waves of adjacent tiles running at
        // the same time meet their shared lines in L2 before eviction.
        constexpr int NS = 4;
        int nbs[7], c0s[3];
        nbs[0] = mycell;
#pragma unroll
        for (int s = 1; s < NS; ++s) nbs[s] = L.up[(size_t)(s - 1) * L.n + mycell];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            c0s[ax] = L.lo[(size_t)ax * L.n + mycell];
            nbs[NS + ax] = c0s[ax] >= 0 ? c0s[ax] : mycell;
        }
        v4f u[7][2];
        if constexpr (!VB) {
#pragma unroll
            for (int k = 0; k < 7; ++k) load_seg(nbs[k], u[k][0], u[k][1]);
        }
        constexpr int P0 = ax_cell_planes(B), TP = ax_tile_planes(B, 3);
        // the transposed lower-face blocks are requested up front as well:
        // 4 consecutive cells share each of their cache lines
        float alo[3][B];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int c0 = c0s[ax], cs = nbs[NS + ax];
            const int t0 = cs / TC, l0 = cs - t0 * TC;
            const float* At = L.vals + ((size_t)t0 * TP + P0 + ax * B + row) * TR + (size_t)l0 * B;
#pragma unroll
            for (int q = 0; q < B; ++q) alo[ax][q] = c0 >= 0 ? At[q] : 0.f;
        }
        const float* __restrict__ A = L.vals + (size_t)tile * TP * TR + threadIdx.x;
        // the cell block's row in column order (the matrix cores take one
        // column per step): plane k gives columns row + k and row - k, which
        // the lane places in a private LDS row (stride 9 against conflicts)
        __shared__ float arow[kWG * 9];
        float a0[B];
        {
            float* w = arow + threadIdx.x * 9;
#pragma unroll
            for (int k = 0; k < P0; ++k) {
                const int jp = row + k >= B ? row + k - B : row + k;
                w[jp] = A[(size_t)k * TR];
                if (k > 0 && 2 * k != B) {
                    const int jm = row >= k ? row - k : row - k + B;
                    w[jm] = A[(ptrdiff_t)k * TR + (jm - row)];
                }
            }
#pragma unroll
            for (int j = 0; j < B; ++j) a0[j] = w[j];
        }
        if constexpr (VB) load_seg(nbs[0], u[0][0], u[0][1]);
        mma_seg(a0, u[0][0], u[0][1]);
#pragma unroll
        for (int s = 1; s < NS; ++s) {
            float a[B];
#pragma unroll
            for (int j = 0; j < B; ++j) a[j] = A[(size_t)(P0 + (s - 1) * B + j) * TR];
            if constexpr (VB) load_seg(nbs[s], u[s][0], u[s][1]);
            mma_seg(a, u[s][0], u[s][1]);
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if constexpr (VB) load_seg(nbs[NS + ax], u[NS + ax][0], u[NS + ax][1]);
            mma_seg(alo[ax], u[NS + ax][0], u[NS + ax][1]);
        }
    } else {
        const int s0 = L.slot_ptr[tile], ns = L.slot_ptr[tile + 1] - s0;
        const float* __restrict__ A = L.vals + (size_t)s0 * B * TR + threadIdx.x;
        const int32_t* __restrict__ nbp = L.snb + (size_t)s0 * TC + lc;
        for (int s = 0; s < ns; ++s) {
            const int nb = nbp[(size_t)s * TC];
            float a[B];
#pragma unroll
            for (int j = 0; j < B; ++j) a[j] = A[((size_t)s * B + j) * TR];
            mma(a, nb);
        }
    }
    __shared__ float ys[kWG * R];
    {
        const int blk = lane >> 2;
        const int rbase = ((threadIdx.x >> 6) * 8 + (blk >> 1)) * B + 4 * (blk & 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ys[(rbase + i) * R + jj] = acc0[i];
            ys[(rbase + i) * R + 4 + jj] = acc1[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = ys[threadIdx.x * R + q];
}

// The Chebyshev step for FP32 8x8 blocks and 8 columns with the block
// product on the matrix cores.
template <bool AX>
__global__ __launch_bounds__(kWG) void k_cheb_step_mfma8(LevelArgs<float> L, const float* __restrict__ d,
                                                         float* __restrict__ x, float* __restrict__ r,
                                                         float* __restrict__ dn, float cd, float cr,
                                                         int assign, int last) {
    constexpr int B = 8, R = 8;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lc = threadIdx.x / B;
    const int cell = tile * Tile<float, 8>::TC + lc;
    float acc[R];
    mfma8_tile_product<AX, false>(L, tile, d, nullptr, acc);
    if (cell >= L.n) return;
    cheb_epilogue_m<float, R>(L, cell * B + (threadIdx.x - lc * B), acc, d, x, r, dn, cd, cr, assign,
                              last);
}

// First sweep from x = 0 on R columns: r = b, d = dinv * b * c1.
template <typename T, int R>
__global__ __launch_bounds__(kWG) void k_cheb_init0_m(int64_t NR, const T* __restrict__ b,
                                                      const T* __restrict__ dinv, T* __restrict__ r,
                                                      T* __restrict__ d, T c1) {
    const int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (k >= NR) return;
    const T v = b[k];
    r[k] = v;
    d[k] = dinv[k / R] * v * c1;
}

template <typename T, int B, int R>
__global__ __launch_bounds__(kWG) void k_restrict_sum_m(int32_t nC, const int32_t* __restrict__ cptr,
                                                        const int32_t* __restrict__ clist,
                                                        const T* __restrict__ rp, T* __restrict__ rc) {
    const int t = blockIdx.x * kWG + threadIdx.x;
    const int K = t / (B * R);
    if (K >= nC) return;
    const int jr = t - K * B * R;           // (j, r) within the coarse cell
    T acc = 0;
    for (int c = cptr[K]; c < cptr[K + 1]; ++c) acc += rp[(size_t)clist[c] * B * R + jr];
    rc[t] = acc;
}

template <typename T, int B, int R>
__global__ __launch_bounds__(kWG) void k_prolong_add_m(int32_t n, const int32_t* __restrict__ parent,
                                                       const T* __restrict__ P, const T* __restrict__ xc,
                                                       const T* __restrict__ dc, T* __restrict__ x,
                                                       const int32_t* __restrict__ ptype) {
    constexpr int TC = Tile<T, B>::TC, TR = Tile<T, B>::TR;
    const int tile = blockIdx.x;
    const int lc = threadIdx.x / B;
    const int e = tile * TC + lc;
    if (lc >= TC || e >= n) return;
    const int i = threadIdx.x - lc * B;
    const int t = e * B + i;
    const int K = parent[e];
    const T* Pe = ptype ? P + (size_t)ptype[e] * B * B + i : P + (size_t)tile * B * TR + threadIdx.x;
    const size_t js = ptype ? B : TR;
    const T* v = xc + (size_t)K * B * R;
    const T* w = dc ? dc + (size_t)K * B * R : nullptr;
    T acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0;
#pragma unroll 8
    for (int j = 0; j < B; ++j) {
        const T p = Pe[j * js];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] += p * (w ? v[j * R + q] + w[j * R + q] : v[j * R + q]);
    }
    T* xp = x + (size_t)t * R;
    T xv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) xv[q] = xp[q];
#pragma unroll
    for (int q = 0; q < R; ++q) xp[q] = xv[q] + acc[q];
}

// X = Ainv Rhs for R columns (row-per-wave, right-hand sides staged in LDS),
// each column summed in the single-column kernel's order for an FP64 Ainv
// (TA = double; an FP32 Ainv is summed in 4 partial sums here, 8 there).
constexpr int kCoarseChunkM = 512;
template <typename Tin, typename Tout, int R, typename TA>
__global__ __launch_bounds__(kWG) void k_coarse_solve_m(int32_t n, const TA* __restrict__ Ainv,
                                                        const Tin* __restrict__ rin,
                                                        Tout* __restrict__ x) {
    __shared__ double rs[kCoarseChunkM * R];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kWG / 64) + wave;
    double s[4][R];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) s[u][q] = 0.0;
    for (int c0 = 0; c0 < n; c0 += kCoarseChunkM) {
        const int len = min(kCoarseChunkM, n - c0);
        __syncthreads();
        for (int k = threadIdx.x; k < len * R; k += kWG) rs[k] = (double)rin[(size_t)c0 * R + k];
        __syncthreads();
        if (row < n) {
            const TA* a = Ainv + (size_t)row * n + c0;
            int c = lane;
            for (; c + 192 < len; c += 256) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double av = (double)a[c + 64 * u];
#pragma unroll
                    for (int q = 0; q < R; ++q) s[u][q] += av * rs[(c + 64 * u) * R + q];
                }
            }
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int cc = c + 64 * u;
                if (cc < len) {
                    const double av = (double)a[cc];
#pragma unroll
                    for (int q = 0; q < R; ++q) s[u][q] += av * rs[cc * R + q];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        double v = (s[0][q] + s[1][q]) + (s[2][q] + s[3][q]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0 && row < n) x[(size_t)row * R + q] = (Tout)v;
    }
}

// Pointwise kernels on N x R column-minor vectors: workgroup g covers the
// kWG*R consecutive entries starting at g*kWG*R; thread x handles entries
// x + q*kWG (q < R), all in column x % R, so every load instruction of a
// wave is contiguous and each thread accumulates a single column.

// Column sums of one value per thread (column threadIdx.x % R) into
// partial[blockIdx.x * R + c].
template <int R>
__device__ __forceinline__ void wg_colsum_store(double v, double* partial) {
    __shared__ double red[kWG / 64][R];
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane < R) red[wv][lane] = v;
    __syncthreads();
    if ((int)threadIdx.x < R) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k][threadIdx.x];
        partial[(size_t)blockIdx.x * R + threadIdx.x] = s;
    }
}

// per-column partial dots of column-minor vectors
template <int R>
__global__ __launch_bounds__(kWG) void k_dot_m(int64_t N, const double* __restrict__ a,
                                               const double* __restrict__ b, double* __restrict__ partial) {
    const int64_t NR = N * R, base = (int64_t)blockIdx.x * kWG * R + threadIdx.x;
    double av[R], bv[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t k = base + (int64_t)q * kWG;
        av[q] = k < NR ? a[k] : 0.0;
        bv[q] = k < NR ? b[k] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) v += av[q] * bv[q];
    wg_colsum_store<R>(v, partial);
}

// Column sums of R partials into sc[slot*R + r]; mode 1/2 as the single
// column kernel (gamma update with beta into sc[4*R + r]).
template <int R>
__global__ __launch_bounds__(kWG) void k_finalize_m(int32_t np, const double* __restrict__ partial,
                                                    double* __restrict__ sc, int slot, int mode) {
    __shared__ double red[kWG][R + 1];
    // four independent running sums per column keep 4 R loads in flight
    constexpr int U = 4;
    double a[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) a[u][q] = 0.0;
    int k = threadIdx.x;
    for (; k + (U - 1) * kWG < np; k += U * kWG) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < R; ++q) a[u][q] += partial[(size_t)(k + u * kWG) * R + q];
    }
    for (; k < np; k += kWG) {
#pragma unroll
        for (int q = 0; q < R; ++q) a[0][q] += partial[(size_t)k * R + q];
    }
    double s[R];
#pragma unroll
    for (int q = 0; q < R; ++q) s[q] = (a[0][q] + a[1][q]) + (a[2][q] + a[3][q]);
#pragma unroll
    for (int q = 0; q < R; ++q) red[threadIdx.x][q] = s[q];
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < R; ++q) red[threadIdx.x][q] += red[threadIdx.x + w][q];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < R) {
        const int q = threadIdx.x;
        const double v = red[0][q];
        if (mode == 0) {
            sc[slot * R + q] = v;
        } else {
            const double g = sc[1 * R + q];
            sc[4 * R + q] = g != 0.0 ? (mode == 1 ? v : v - sc[5 * R + q]) / g : 0.0;
            sc[slot * R + q] = v;
            sc[1 * R + q] = v;
        }
    }
}

// x += alpha_c p, r -= alpha_c q for active columns c; per-column ||r||^2.
template <int R>
__global__ __launch_bounds__(kWG) void k_update_xr_m(int64_t N, const double* __restrict__ sc,
                                                     const int* __restrict__ active,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ partial) {
    const int64_t NR = N * R, base = (int64_t)blockIdx.x * kWG * R + threadIdx.x;
    const int c = threadIdx.x % R;
    const double alpha = active[c] ? sc[1 * R + c] / sc[2 * R + c] : 0.0;
    double pv[R], qv[R], xv[R], rv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int64_t k = base + (int64_t)u * kWG;
        const bool in = k < NR;
        pv[u] = in ? p[k] : 0.0;
        qv[u] = in ? q[k] : 0.0;
        xv[u] = in ? x[k] : 0.0;
        rv[u] = in ? r[k] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int64_t k = base + (int64_t)u * kWG;
        const double rn = rv[u] - alpha * qv[u];
        if (k < NR) {
            x[k] = xv[u] + alpha * pv[u];
            r[k] = rn;
            v += rn * rn;
        }
    }
    wg_colsum_store<R>(v, partial);
}

template <int R>
__global__ __launch_bounds__(kWG) void k_update_p_m(int64_t NR, const double* __restrict__ sc,
                                                    const double* __restrict__ z, double* __restrict__ p,
                                                    int first) {
    const int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (k >= NR) return;
    p[k] = first ? z[k] : z[k] + sc[4 * R + (k % R)] * p[k];
}

// Load vector on R columns: f = cU hist + iapp - chi g, b = M_K f per column.
template <int B, int R>
__global__ __launch_bounds__(256) void k_rhs_m(int32_t n, IonicParams P, double cU,
                                               const double* __restrict__ mass, const double* U,
                                               const double* Up, const double* __restrict__ iapp,
                                               const double* __restrict__ g, double* __restrict__ b,
                                               double* xout) {
    __shared__ double f[256 * R];
    const int cells_per = blockDim.x / B;
    const int lc = threadIdx.x / B, i = threadIdx.x - lc * B;
    const int cell = blockIdx.x * cells_per + lc;
    const bool act = lc < cells_per && cell < n;
    const int64_t t = (int64_t)cell * B + i;
    double u[R];
    if (act) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const size_t k = (size_t)t * R + q;
            u[q] = U[k];
            const double hist = P.bdf == 2 ? 4.0 * u[q] - Up[k] : u[q];
            f[threadIdx.x * R + q] = cU * hist + (iapp ? iapp[k] : 0.0) - P.chi * g[k];
        }
    }
    __syncthreads();
    if (!act) return;
    const double* M = mass + (size_t)cell * ((B * B + 1) / 2 * 2) + i;
    double acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
#pragma unroll 8
    for (int j = 0; j < B; ++j) {
        const double m = M[j * B];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] += m * f[(lc * B + j) * R + q];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const size_t k = (size_t)t * R + q;
        b[k] = acc[q];
        if (xout) xout[k] = u[q];
    }
}

}  // namespace dgmg
