// gfx950 HIP kernels of the per-step path.  Included by solver.hip only.
//
// Layout on the device (one level, scalar type T = double or float):
//  * vectors: cell-major, DoF (K, i) at K*B + i;
//  * cell blocks diag[K] and face blocks fblk[f] are B x B and stored
//    column-major (entry (i, j) at j*B + i) so that the B lanes owning the
//    rows of one cell read consecutive addresses for every column j;
//  * face f couples plus cell (rows) and minus cell (columns); the plus side
//    applies F, the minus side applies F^T from the same stored block (A is
//    symmetric, section 3), so every face block is stored once;
//  * cell -> neighbour lists (CSR) hold the neighbour cell and
//    (face << 1 | side), side 1 meaning "this cell is the minus side";
//  * prolongation blocks P_e (fine node i, coarse function j) column-major.
// One thread owns one DoF row.  Workgroups are mapped XCD-aware: the 8 XCDs
// receive consecutive workgroup ids round-robin, so tile = (id % 8) * per +
// id / 8 gives each XCD a contiguous range of cells and keeps the second
// read of a face block (by the neighbour) in that XCD's L2 where possible.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgmg {

constexpr int kWG = 256;

__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
    // bijective remap of [0, nblk): XCD x = bid % 8 gets tiles [x*q + min(x,r), ...)
    const int x = bid & 7, k = bid >> 3;
    const int q = nblk >> 3, r = nblk & 7;
    return x * q + (x < r ? x : r) + k;
}

template <typename T>
struct LevelArgs {
    const T* __restrict__ diag;
    const T* __restrict__ fblk;
    const T* __restrict__ dinv;
    const int32_t* __restrict__ nbr_ptr;
    const int32_t* __restrict__ nbr_cell;
    const int32_t* __restrict__ nbr_code;
    int32_t n;
};

// (A v)[cell, i] with v = va + vb (vb may be null).
template <typename T, int B>
__device__ __forceinline__ T row_apply(const LevelArgs<T>& L, int cell, int i,
                                       const T* __restrict__ va, const T* __restrict__ vb) {
    constexpr int BB = B * B;
    T acc = 0;
    {
        const T* D = L.diag + (size_t)cell * BB + i;
        const T* v = va + (size_t)cell * B;
        if (vb) {
            const T* w = vb + (size_t)cell * B;
#pragma unroll
            for (int j = 0; j < B; ++j) acc += D[j * B] * (v[j] + w[j]);
        } else {
#pragma unroll
            for (int j = 0; j < B; ++j) acc += D[j * B] * v[j];
        }
    }
    const int e0 = L.nbr_ptr[cell], e1 = L.nbr_ptr[cell + 1];
    for (int e = e0; e < e1; ++e) {
        const int nb = L.nbr_cell[e];
        const int code = L.nbr_code[e];
        const T* F = L.fblk + (size_t)(code >> 1) * BB;
        const T* v = va + (size_t)nb * B;
        const T* w = vb ? vb + (size_t)nb * B : nullptr;
        if ((code & 1) == 0) {
            F += i;  // row i of F: entries at j*B + i
            if (w) {
#pragma unroll
                for (int j = 0; j < B; ++j) acc += F[j * B] * (v[j] + w[j]);
            } else {
#pragma unroll
                for (int j = 0; j < B; ++j) acc += F[j * B] * v[j];
            }
        } else {
            F += (size_t)i * B;  // row i of F^T = column i of F: contiguous
            if (w) {
#pragma unroll
                for (int j = 0; j < B; ++j) acc += F[j] * (v[j] + w[j]);
            } else {
#pragma unroll
                for (int j = 0; j < B; ++j) acc += F[j] * v[j];
            }
        }
    }
    return acc;
}

// Workgroup sum of a double into partial[blockIdx.x] (deterministic order).
__device__ __forceinline__ void wg_sum_store(double v, double* partial) {
    __shared__ double red[kWG / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
        partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------- apply
// y = A (va + vb); optional partial of dot(w, y).
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_apply(LevelArgs<T> L, const T* __restrict__ va,
                                               const T* __restrict__ vb, T* __restrict__ y,
                                               const T* __restrict__ w, double* __restrict__ partial) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = tile * kWG + threadIdx.x;
    const int cell = t / B, i = t - cell * B;
    double contrib = 0.0;
    if (cell < L.n) {
        const T a = row_apply<T, B>(L, cell, i, va, vb);
        y[t] = a;
        if (w) contrib = (double)w[t] * (double)a;
    }
    if (partial) wg_sum_store(contrib, partial);
}

// Residual: r = rhs - A (va + vb); optional d = dinv * r * c1, x_out = va + vb,
// partial of ||r||^2.
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_residual(LevelArgs<T> L, const T* __restrict__ va,
                                                  const T* __restrict__ vb, const T* __restrict__ rhs,
                                                  T* __restrict__ r, T* __restrict__ d, T c1,
                                                  T* __restrict__ xout, double* __restrict__ partial) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = tile * kWG + threadIdx.x;
    const int cell = t / B, i = t - cell * B;
    double contrib = 0.0;
    if (cell < L.n) {
        const T a = row_apply<T, B>(L, cell, i, va, vb);
        const T rr = rhs[t] - a;
        r[t] = rr;
        if (d) d[t] = L.dinv[t] * rr * c1;
        if (xout) xout[t] = vb ? va[t] + vb[t] : va[t];
        contrib = (double)rr * (double)rr;
    }
    if (partial) wg_sum_store(contrib, partial);
}

// One inner Chebyshev step (gather vector d):
//   x += d (x = d when assign), r -= A d, dn = cd * d + cr * dinv * r.
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_cheb_step(LevelArgs<T> L, const T* __restrict__ d,
                                                   T* __restrict__ x, T* __restrict__ r,
                                                   T* __restrict__ dn, T cd, T cr, int assign) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = tile * kWG + threadIdx.x;
    const int cell = t / B, i = t - cell * B;
    if (cell >= L.n) return;
    const T a = row_apply<T, B>(L, cell, i, d, nullptr);
    const T dt = d[t];
    x[t] = assign ? dt : x[t] + dt;
    const T rr = r[t] - a;
    r[t] = rr;
    dn[t] = cd * dt + cr * L.dinv[t] * rr;
}

// First sweep from x = 0: r = b, d = dinv * b * c1.
template <typename T>
__global__ __launch_bounds__(kWG) void k_cheb_init0(int64_t N, const T* __restrict__ b,
                                                    const T* __restrict__ dinv, T* __restrict__ r,
                                                    T* __restrict__ d, T c1) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= N) return;
    const T v = b[t];
    r[t] = v;
    d[t] = dinv[t] * v * c1;
}

// ----------------------------------------------------------- transfers
// Restriction rc[K, j] = sum_{e child of K} sum_i P_e(i, j) r[e, i].
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_restrict(int32_t nC, const int32_t* __restrict__ cptr,
                                                  const int32_t* __restrict__ clist,
                                                  const T* __restrict__ P, const T* __restrict__ r,
                                                  T* __restrict__ rc) {
    const int t = blockIdx.x * kWG + threadIdx.x;
    const int K = t / B, j = t - K * B;
    if (K >= nC) return;
    T acc = 0;
    const int c0 = cptr[K], c1 = cptr[K + 1];
    for (int c = c0; c < c1; ++c) {
        const int e = clist[c];
        const T* Pe = P + (size_t)e * B * B + (size_t)j * B;  // column j, contiguous in i
        const T* re = r + (size_t)e * B;
#pragma unroll
        for (int i = 0; i < B; ++i) acc += Pe[i] * re[i];
    }
    rc[t] = acc;
}

// Prolongation with correction: x[e, i] += sum_j P_e(i, j) (xc + dc)[parent(e), j].
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_prolong_add(int32_t n, const int32_t* __restrict__ parent,
                                                     const T* __restrict__ P, const T* __restrict__ xc,
                                                     const T* __restrict__ dc, T* __restrict__ x) {
    const int t = blockIdx.x * kWG + threadIdx.x;
    const int e = t / B, i = t - e * B;
    if (e >= n) return;
    const int K = parent[e];
    const T* Pe = P + (size_t)e * B * B + i;
    const T* v = xc + (size_t)K * B;
    T acc = 0;
    if (dc) {
        const T* w = dc + (size_t)K * B;
#pragma unroll
        for (int j = 0; j < B; ++j) acc += Pe[j * B] * (v[j] + w[j]);
    } else {
#pragma unroll
        for (int j = 0; j < B; ++j) acc += Pe[j * B] * v[j];
    }
    x[t] += acc;
}

// ------------------------------------------------------------ coarse
// Split-K dense GEMV with the symmetric coarse inverse (row-major, FP64):
// partial[chunk][col] = sum_{rows in chunk} Ainv[row][col] * r[row].
template <typename Tin>
__global__ __launch_bounds__(kWG) void k_coarse_gemv(int32_t n, int32_t rows_per_chunk,
                                                     const double* __restrict__ Ainv,
                                                     const Tin* __restrict__ r,
                                                     double* __restrict__ partial) {
    const int col = blockIdx.x * kWG + threadIdx.x;
    const int chunk = blockIdx.y;
    const int r0 = chunk * rows_per_chunk;
    const int r1 = min(n, r0 + rows_per_chunk);
    if (col >= n) return;
    double acc = 0.0;
    for (int row = r0; row < r1; ++row) acc += Ainv[(size_t)row * n + col] * (double)r[row];
    partial[(size_t)chunk * n + col] = acc;
}

template <typename Tout>
__global__ __launch_bounds__(kWG) void k_coarse_reduce(int32_t n, int32_t nchunk,
                                                       const double* __restrict__ partial,
                                                       Tout* __restrict__ x) {
    const int col = blockIdx.x * kWG + threadIdx.x;
    if (col >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += partial[(size_t)c * n + col];
    x[col] = (Tout)s;
}

// ------------------------------------------------------------ vectors
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kWG) void k_cast(int64_t N, const Tin* __restrict__ a,
                                              const Tin* __restrict__ b, Tout* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= N) return;
    out[t] = b ? (Tout)((double)a[t] + (double)b[t]) : (Tout)a[t];
}

// partial dots: (a, b) and optionally (a, c)
__global__ __launch_bounds__(kWG) void k_dot(int64_t N, const double* __restrict__ a,
                                             const double* __restrict__ b,
                                             double* __restrict__ partial) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (t < N) v = a[t] * b[t];
    wg_sum_store(v, partial);
}

// Final reduction of partials into sc[slot]; mode 1 also forms
// beta = value / sc[1] into sc[4] and moves value into sc[1] (gamma update);
// mode 2 (flexible) uses sc[5] = (r_new, z_old): beta = (value - sc[5]) / sc[1].
__global__ __launch_bounds__(kWG) void k_finalize(int32_t np, const double* __restrict__ partial,
                                                  double* __restrict__ sc, int slot, int mode) {
    __shared__ double red[kWG];
    double s = 0.0;
    for (int k = threadIdx.x; k < np; k += kWG) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0];
        if (mode == 0) {
            sc[slot] = v;
        } else {
            const double beta = (mode == 1 ? v : v - sc[5]) / sc[1];
            sc[4] = beta;
            sc[slot] = v;
            sc[1] = v;
        }
    }
}

// x += alpha p; r -= alpha q with alpha = sc[1] / sc[2]; partial ||r||^2.
__global__ __launch_bounds__(kWG) void k_update_xr(int64_t N, const double* __restrict__ sc,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ partial) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const double alpha = sc[1] / sc[2];
    double v = 0.0;
    if (t < N) {
        x[t] += alpha * p[t];
        const double rn = r[t] - alpha * q[t];
        r[t] = rn;
        v = rn * rn;
    }
    wg_sum_store(v, partial);
}

// p = z + beta p with beta = sc[4] (or p = z when first).
__global__ __launch_bounds__(kWG) void k_update_p(int64_t N, const double* __restrict__ sc,
                                                  const double* __restrict__ z,
                                                  double* __restrict__ p, int first) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t >= N) return;
    p[t] = first ? z[t] : z[t] + sc[4] * p[t];
}

}  // namespace dgmg
