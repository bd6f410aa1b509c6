// gfx950 HIP kernels of the per-step path.  Included by solver.hip only.
//
// Layout on the device (one level, scalar type T = double or float):
//  * vectors: cell-major, DoF (K, i) at K*B + i;
//  * operator: "tile-ELL".  Cells are grouped in tiles of TC = 256/B cells
//    (one workgroup, thread = (cell in tile, row i)).  Tile t owns ns_t slots
//    (its cell blocks, then one slot per neighbour entry, ns_t = 1 + largest
//    neighbour count in the tile); slot s holds, for every cell of the tile,
//    the B x B block coupling that cell to its s-th column cell, already
//    oriented for the row cell (a face block F for the plus cell, F^T for the
//    minus cell; zero where the cell has fewer neighbours).  Entries are
//    interleaved so that for a fixed (slot, column j) the TC*B rows of the
//    tile are contiguous: vals[(slot*B + j)*TC*B + lc*B + i].  A wave's 64
//    lanes therefore read 64 consecutive values per load.  Each face block is
//    stored twice (once per side): reading a single stored copy transposed
//    from the other side costs more in cache-line traffic than the second
//    copy costs in bytes on this hardware;
//  * "axis-ELL" (fine level of a conforming quad/hex mesh, where every cell
//    has at most one face neighbour per axis direction): tile t holds
//    TP = B/2 + 1 + d*B planes of TR values at a fixed stride -- the
//    symmetric cell blocks in B/2 + 1 cyclic planes (ax_cell_planes below)
//    and, per axis a, B planes of the block U_a(c) = A[c, up_a(c)] of the
//    face on the cell's upper a-side (zero if none), interleaved as above.
//    Each face block is stored once.  The lower a-face of cell c is
//    U_a(lo_a(c)) read transposed: thread (c, i) reads column i of that
//    block, B contiguous values at (tile0*TP + B/2 + 1 + a*B + i)*TR +
//    lc0*B; consecutive cells have consecutive lower neighbours, so a wave's
//    reads stay within a few cache lines per column plane;
//  * prolongation blocks use the same interleaving with one slot per tile.
// Workgroups are mapped XCD-aware: the 8 XCDs receive consecutive workgroup
// ids round-robin, so tile = (id % 8) * per + id / 8 gives each XCD a
// contiguous range of cells (neighbouring tiles share their x gathers in the
// XCD's L2).
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

// Constants of the matrix-free fine level on identical axis-aligned boxes:
// 1D tables on [0,1] (Q = p + 1 Lobatto nodes, Q Gauss points) and the box
// geometry; D points to the per-cell packed (scaled) conductivity.
constexpr int kMfMaxQ = 5;
template <typename T>
struct MfConst {
    T Ig[kMfMaxQ * kMfMaxQ];   // Ig[g*Q + j] = l_j(gauss_g)
    T Dg[kMfMaxQ * kMfMaxQ];   // Dg[g*Q + j] = l_j'(gauss_g)
    T Ed[2 * kMfMaxQ];         // Ed[e*Q + j] = l_j'(e), e = 0, 1 (l_j(e) is 0 or 1: Lobatto ends)
    T gw[kMfMaxQ];             // Gauss weights on [0,1]
    T hinv[3];                 // 1 / h_k
    T vol;                     // |K|
    T area[3];                 // |F| of a face normal to axis k
    T eta[3];                  // penalty factor of a face normal to axis k
    T cM;                      // mass coefficient of A_0
    const T* D;                // per cell: packed symmetric D (d(d+1)/2 values)
};

template <typename T>
struct LevelArgs {
    const T* __restrict__ vals;            // tile-ELL or axis-ELL blocks
    const int32_t* __restrict__ slot_ptr;  // tile-ELL: ntiles + 1
    const int32_t* __restrict__ snb;       // tile-ELL: (slot, cell in tile) -> column cell
    const T* __restrict__ dinv;
    int32_t n;
    const int32_t* __restrict__ up;        // axis-ELL: [d][n] upper neighbour (itself if none)
    const int32_t* __restrict__ lo;        // axis-ELL: [d][n] lower neighbour (-1 if none)
    MfConst<T> mf;                         // matrix-free fine level (layout 2)
    const int32_t* __restrict__ cmap;      // tile-ELL: tile position -> cell (null: identity)
};

// spatial dimension of a block size (Q1..Q3 in 2D: 4, 9, 16; in 3D: 8, 27, 64)
template <int B>
constexpr int dim_of() {
    return (B == 8 || B == 27 || B == 64) ? 3 : 2;
}

template <typename T, int B>
struct Tile {
    static constexpr int TC = kWG / B;   // cells per tile / workgroup
    static constexpr int TR = TC * B;    // rows per tile
};

// Axis-ELL storage of a cell's diagonal block, which is symmetric: plane k
// (k = 0 .. b/2) holds at the tile row of (cell, i) the entry
// A_K[i][(i + k) mod b].  Every pair {i, j} is stored once (both orders when
// b is even and j - i = b/2), so the block takes b/2 + 1 planes instead of b.
// Row i reads column (i - k) mod b from plane k at row (i - k) mod b of the
// same cell: the same cache lines as the plane's own entries.  The d upper
// face blocks follow with b planes each.
constexpr int ax_cell_planes(int b) { return b / 2 + 1; }
constexpr int ax_tile_planes(int b, int d) { return ax_cell_planes(b) + d * b; }

// Sparse face blocks of a nodal fine level (section 3: the face terms of a_h
// test and trial traces, and a Q_p Lagrange function on Gauss-Lobatto nodes
// has a nonzero trace on a face only if its node lies on that face).  Entry
// (i, j) of the block A[c, up_a(c)] therefore vanishes unless node i lies on
// the upper a-face of c or node j on the lower a-face of the neighbour: with
// q nodes per axis, nF = b / q of the b rows and columns.  Per axis the
// block is stored as nF full planes (the columns j on the lower face, by
// tangential index) and b - nF sparse planes (the other columns, ordered by
// (tangential index, coordinate - 1); each holds only the nF rows on the
// upper face: TC nF values, by cell slot then the row's tangential index).
__host__ __device__ constexpr int ax_nodes_1d(int b, int d) { return d == 2 ? (b == 4 ? 2 : b == 9 ? 3 : b == 16 ? 4 : 5) : (b == 8 ? 2 : b == 27 ? 3 : 4); }
// coordinate of node j along axis a, and its index among the nodes of a face normal to a
__host__ __device__ constexpr int node_coord(int j, int a, int q) { return a == 0 ? j % q : a == 1 ? (j / q) % q : j / (q * q); }
__host__ __device__ constexpr int node_tan(int j, int a, int q) {
    return a == 0 ? (j / q) % q + q * (j / (q * q)) : a == 1 ? j % q + q * (j / (q * q)) : j % (q * q);
}
// values per axis and per tile of the sparse-face axis layout (tiles of tc cells)
constexpr int64_t ax_sparse_axis_values(int b, int d, int tc) {
    return (int64_t)(b / ax_nodes_1d(b, d)) * tc * b + (int64_t)(b - b / ax_nodes_1d(b, d)) * tc * (b / ax_nodes_1d(b, d));
}
constexpr int64_t ax_sparse_tile_values(int b, int d, int tc) {
    return (int64_t)ax_cell_planes(b) * tc * b + d * ax_sparse_axis_values(b, d, tc);
}

// Slots whose loads are issued together before any of them is accumulated
// (bounded so that G*B values stay in registers): all five slots of a 2D
// quad cell for B <= 9, fewer for larger blocks.
template <int B>
constexpr int slot_group() {
    return (48 / B) < 1 ? 1 : ((48 / B) > 5 ? 5 : (48 / B));
}

// Block sizes whose cells the block layouts keep inside one wave: lane l of
// wave w holds row l % B of tile cell w (64/B) + l / B, the lanes past
// (64/B) B stay idle, and the tile keeps its 256/B cells.  A cell's B lanes
// then share gathered vector values by lane shuffles (ds_bpermute, the LDS
// crossbar) instead of each loading all B values through the address unit.
template <int B>
constexpr bool whole_wave_cells() {
    return B == 4 || B == 8 || B == 9 || B == 16 || B == 64;
}
static_assert(4 * (64 / 9) == 256 / 9 && 4 * (64 / 8) == 256 / 8, "wave-aligned tiles keep 256/B cells");

// (A v) at row (tile*TC + lc, i) of the tile's thread (lc, i), v = va (+ vb
// when VB).  Loads of a group of G slots -- block values and the gathered
// vector segments -- are all issued before the group is accumulated; slots
// past a count reload a valid slot (cache hit) and are skipped.
template <typename T, int B, bool VB>
__device__ __forceinline__ void gather_group(const T* __restrict__ va, const T* __restrict__ vb,
                                             int nb, T* v) {
    const T* x = va + (size_t)nb * B;
    if constexpr (VB) {
        const T* y = vb + (size_t)nb * B;
#pragma unroll
        for (int j = 0; j < B; ++j) v[j] = x[j] + y[j];
    } else {
#pragma unroll
        for (int j = 0; j < B; ++j) v[j] = x[j];
    }
}

// The lane's own element of cell nb's segment: (va + vb)[nb B + i].
template <typename T, int B, bool VB>
__device__ __forceinline__ T gather_own(const T* __restrict__ va, const T* __restrict__ vb, int nb,
                                        int i) {
    const size_t k = (size_t)nb * B + i;
    if constexpr (VB)
        return va[k] + vb[k];
    else
        return va[k];
}

// v[j] = the element of lane base + j (whole-wave cells: the cell's B lanes
// hold one segment between them).
template <typename T, int B>
__device__ __forceinline__ void share_segment(T x, int base, T* v) {
#pragma unroll
    for (int j = 0; j < B; ++j) v[j] = __shfl(x, base + j, 64);
}

template <typename T, int B, bool VB, bool WW>
__device__ __forceinline__ T ell_row_apply(const LevelArgs<T>& L, int tile, int lc, int ri, int i,
                                           const T* __restrict__ va, const T* __restrict__ vb) {
    constexpr int TC = Tile<T, B>::TC, TR = Tile<T, B>::TR, G = slot_group<B>();
    const int s0 = L.slot_ptr[tile], ns = L.slot_ptr[tile + 1] - s0;
    const int base = ((int)threadIdx.x & 63) - i;   // lane of the cell's row 0 (whole-wave cells)
    const T* __restrict__ A = L.vals + (size_t)s0 * B * TR + ri;
    const int32_t* __restrict__ nbp = L.snb + (size_t)s0 * TC + lc;
    T acc = 0;
    for (int g = 0; g < ns; g += G) {
        int nbq[G];
        T a[G][B], v[G][B];
#pragma unroll
        for (int q = 0; q < G; ++q) nbq[q] = nbp[(size_t)min(g + q, ns - 1) * TC];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const T* As = A + (size_t)min(g + q, ns - 1) * B * TR;
#pragma unroll
            for (int j = 0; j < B; ++j) a[q][j] = As[(size_t)j * TR];
        }
        if constexpr (WW) {
            T xq[G];
#pragma unroll
            for (int q = 0; q < G; ++q) xq[q] = gather_own<T, B, VB>(va, vb, nbq[q], i);
#pragma unroll
            for (int q = 0; q < G; ++q) share_segment<T, B>(xq[q], base, v[q]);
        } else {
#pragma unroll
            for (int q = 0; q < G; ++q) gather_group<T, B, VB>(va, vb, nbq[q], v[q]);
        }
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (g + q < ns) {
#pragma unroll
                for (int j = 0; j < B; ++j) acc += a[q][j] * v[q][j];
            }
    }
    return acc;
}

// The same row product on the axis-ELL layout: the d upper face slots in
// groups as above, the cell block from its b/2 + 1 symmetric planes (the
// cell's own vector values in the matching cyclic order), then each lower
// face as the transposed column of the neighbour's stored block.
// SF: sparse face blocks (see ax_sparse_tile_values).
template <typename T, int B, bool VB, bool WW, bool SF = false>
__device__ __forceinline__ T ax_row_apply(const LevelArgs<T>& L, int tile, int cell, int ri, int i,
                                          const T* __restrict__ va, const T* __restrict__ vb) {
    constexpr int TC = Tile<T, B>::TC, TR = Tile<T, B>::TR, D = dim_of<B>();
    constexpr int P0 = ax_cell_planes(B), TP = ax_tile_planes(B, D);
    constexpr int Q = ax_nodes_1d(B, D), NFN = B / Q, SP = TC * NFN;
    constexpr int64_t AXS = ax_sparse_axis_values(B, D, TC);
    constexpr int64_t TSTRIDE = SF ? ax_sparse_tile_values(B, D, TC) : (int64_t)TP * TR;
    constexpr int G = slot_group<B>() < D ? slot_group<B>() : D;
    // cell-block planes per load group (FP64: fewer, to keep 8 waves per SIMD)
    constexpr int KG = B > 27 ? 8 : (sizeof(T) == 8 ? 3 : P0);
    const int base = ((int)threadIdx.x & 63) - i;   // lane of the cell's row 0 (whole-wave cells)
    const T* __restrict__ A = L.vals + (size_t)tile * TSTRIDE + ri;
    // lower neighbours first: their blocks and values are the longest chain
    int lo_nb[D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) lo_nb[ax] = L.lo[(size_t)ax * L.n + cell];
    T acc = 0;
    // cell block: plane k holds A[i][i+k] at row i.  Row i takes it times
    // x[i+k]; the symmetric entry A[i][i-k] is the plane's value at row i-k,
    // so row i-k's product A[i-k][i] x[i-k] is what row i needs from it:
    // whole-wave cells hand it over by a lane shuffle, other cells read the
    // entry at the mirrored row (same cache lines) and the column value
    {
        T xself = 0;
        if constexpr (WW) xself = gather_own<T, B, VB>(va, vb, cell, i);
#pragma unroll
        for (int k0 = 0; k0 < P0; k0 += KG) {
            T ao[KG], t1[KG], t2[KG];
#pragma unroll
            for (int q = 0; q < KG; ++q) {
                const int k = k0 + q;
                if (k >= P0) break;
                const int jp = i + k >= B ? i + k - B : i + k;
                const int jm = i >= k ? i - k : i - k + B;
                ao[q] = A[(size_t)k * TR];
                if constexpr (WW) {
                    t1[q] = __shfl(xself, base + jp, 64);
                } else {
                    t1[q] = gather_own<T, B, VB>(va, vb, cell, jp);
                    t2[q] = (k > 0 && 2 * k != B)
                                ? A[(ptrdiff_t)k * TR + (jm - i)] * gather_own<T, B, VB>(va, vb, cell, jm)
                                : T(0);
                }
            }
#pragma unroll
            for (int q = 0; q < KG; ++q) {
                const int k = k0 + q;
                if (k >= P0) break;
                acc += ao[q] * t1[q];
                if (k > 0 && 2 * k != B) {
                    if constexpr (WW) {
                        const int jm = i >= k ? i - k : i - k + B;
                        acc += __shfl(ao[q] * xself, base + jm, 64);
                    } else {
                        acc += t2[q];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < D; g += G) {
        int nbq[G];
        T a[G][B], v[G][B];
#pragma unroll
        for (int q = 0; q < G; ++q) nbq[q] = L.up[(size_t)min(g + q, D - 1) * L.n + cell];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if constexpr (SF) {
                // full planes at the thread's row; sparse planes only on
                // the rows of the upper face, at (cell slot, tangential index)
                const int ax = min(g + q, D - 1);
                const T* As = A + (size_t)P0 * TR + (size_t)ax * AXS;
                const T* Ss = As - ri + (size_t)NFN * TR + (size_t)(ri - i) / B * NFN + node_tan(i, ax, Q);
                const bool on_up = node_coord(i, ax, Q) == Q - 1;
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int cj = node_coord(j, ax, Q), tj = node_tan(j, ax, Q);
                    if (cj == 0) a[q][j] = As[(size_t)tj * TR];
                    else a[q][j] = on_up ? Ss[(size_t)(tj * (Q - 1) + cj - 1) * SP] : T(0);
                }
            } else {
                const T* As = A + (size_t)(P0 + min(g + q, D - 1) * B) * TR;
#pragma unroll
                for (int j = 0; j < B; ++j) a[q][j] = As[(size_t)j * TR];
            }
        }
        if constexpr (WW) {
            T xq[G];
#pragma unroll
            for (int q = 0; q < G; ++q) xq[q] = gather_own<T, B, VB>(va, vb, nbq[q], i);
#pragma unroll
            for (int q = 0; q < G; ++q) share_segment<T, B>(xq[q], base, v[q]);
        } else {
#pragma unroll
            for (int q = 0; q < G; ++q) gather_group<T, B, VB>(va, vb, nbq[q], v[q]);
        }
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (g + q < D) {
#pragma unroll
                for (int j = 0; j < B; ++j) acc += a[q][j] * v[q][j];
            }
    }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        const int c0 = lo_nb[ax];
        if (c0 >= 0) {
            const int t0 = c0 / TC, l0 = c0 - t0 * TC;
            T a[B], v[B];
            if constexpr (SF) {
                // column i of the neighbour's block: a full plane when node i
                // lies on the lower face, else the upper-face rows only
                const T* As = L.vals + (size_t)t0 * TSTRIDE + (size_t)P0 * TR + (size_t)ax * AXS;
                const int ci = node_coord(i, ax, Q), ti = node_tan(i, ax, Q);
                if (ci == 0) {
                    const T* At = As + (size_t)ti * TR + (size_t)l0 * B;
#pragma unroll
                    for (int r = 0; r < B; ++r) a[r] = At[r];
                } else {
                    const T* At = As + (size_t)NFN * TR + (size_t)(ti * (Q - 1) + ci - 1) * SP + (size_t)l0 * NFN;
#pragma unroll
                    for (int r = 0; r < B; ++r)
                        a[r] = node_coord(r, ax, Q) == Q - 1 ? At[node_tan(r, ax, Q)] : T(0);
                }
            } else {
                const T* At = L.vals + ((size_t)t0 * TP + P0 + ax * B + i) * TR + (size_t)l0 * B;
#pragma unroll
                for (int r = 0; r < B; ++r) a[r] = At[r];
            }
            if constexpr (WW)
                share_segment<T, B>(gather_own<T, B, VB>(va, vb, c0, i), base, v);
            else
                gather_group<T, B, VB>(va, vb, c0, v);
#pragma unroll
            for (int r = 0; r < B; ++r) acc += a[r] * v[r];
        }
    }
    return acc;
}

template <typename T, int B, bool VB>
__device__ __forceinline__ T mf_row_apply(const LevelArgs<T>& L, int lc, int cell, bool active,
                                          const T* __restrict__ va, const T* __restrict__ vb,
                                          T** lds_free);

// Operator layouts of a level: tile-ELL, axis-ELL, matrix-free boxes,
// axis-ELL with sparse face blocks (nodal fine levels, single column).
enum { LY_TILE = 0, LY_AXIS = 1, LY_MF = 2, LY_AXS = 3 };

// (A (va + vb)) at the thread's row for layout LY.  The matrix-free product
// synchronises the workgroup, so every thread calls this; rows of inactive
// threads are not used.  When lds_free is given, the matrix-free product
// stores there an LDS region of at least kWG values that no thread reads
// any more (usable by the caller's epilogue without a further barrier).
// ri is the thread's row within the tile (lc B + i), i its row of the cell.
template <typename T, int B, bool VB, int LY>
__device__ __forceinline__ T row_apply(const LevelArgs<T>& L, int tile, int lc, int cell, int ri, int i,
                                       bool active, const T* __restrict__ va, const T* __restrict__ vb,
                                       T** lds_free = nullptr) {
    if constexpr (LY == LY_MF) {
        return mf_row_apply<T, B, VB>(L, lc, cell, active, va, vb, lds_free);
    } else {
        // a cell's lanes are all active or all inactive, so the shuffles of
        // an active cell read active lanes only
        if (!active) return T(0);
        if constexpr (LY == LY_AXIS || LY == LY_AXS)
            return ax_row_apply<T, B, VB, whole_wave_cells<B>(), LY == LY_AXS>(L, tile, cell, ri, i, va, vb);
        else
            return ell_row_apply<T, B, VB, whole_wave_cells<B>()>(L, tile, lc, ri, i, va, vb);
    }
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

// Cell-block Jacobi term of the smoother at the thread's row (i of `cell`):
// z_i = sum_j (D_K^-1)_ij v_j over the cell's rows, with D_K^-1 symmetric and
// row-major per cell (the lanes of a cell read consecutive words of column
// j).  v is the workgroup's row values, staged in LDS here (the matrix-free
// product passes its free region; the block layouts use their own), so every
// thread of the workgroup must call this; inactive threads pass v = 0.
template <typename T, int B, int LY>
__device__ __forceinline__ T block_jacobi_row(const T* __restrict__ Dinv, T v, int lc, int cell, int ri,
                                              int i, bool active, T* lds_free) {
    __shared__ T vs_own[LY == LY_MF ? 1 : kWG];
    T* vs = LY == LY_MF ? lds_free : vs_own;
    if (ri < Tile<T, B>::TR) vs[ri] = v;
    __syncthreads();
    T z = 0;
    if (active) {
        const T* Dc = Dinv + (size_t)cell * B * B + i;
        const T* vc = vs + lc * B;
#pragma unroll
        for (int j = 0; j < B; ++j) z += Dc[(size_t)j * B] * vc[j];
    }
    return z;
}

// ---------------------------------------------------------------- apply
// Thread (tile, lc, i) owns row i of cell tile * TC + lc, or, when MAPPED
// (a tile-ELL level whose tiles group cells of similar neighbour count), of
// cell cmap[tile * TC + lc]; vectors stay in cell order either way.
// With WW (whole-wave cells, block layouts) lane l of wave w holds row
// l % B of tile cell w (64/B) + l / B and the lanes past (64/B) B are idle
// (lc = TC); otherwise thread x holds row x % B of tile cell x / B.  ri is
// the thread's row within the tile (>= TR for idle lanes), ti its row of the
// cell.
#define DGMG_TILE_THREAD_M(T, B, MAPPED, WW)                                                   \
    const int tile = xcd_tile(blockIdx.x, gridDim.x);                                          \
    const int lane_ = (int)threadIdx.x & 63, lcw_ = lane_ / B;                                 \
    const int lc = (WW) ? (lcw_ < 64 / B ? ((int)threadIdx.x >> 6) * (64 / B) + lcw_ : Tile<T, B>::TC) \
                        : (int)threadIdx.x / B;                                                \
    const int ti = (WW) ? lane_ - lcw_ * B : (int)threadIdx.x - lc * B;                        \
    const int ri = lc * B + ti;                                                                \
    const int pos = tile * Tile<T, B>::TC + lc;                                                \
    const bool active = lc < Tile<T, B>::TC && pos < L.n;                                      \
    const int cell = ((MAPPED) && L.cmap && active) ? L.cmap[pos] : pos;                       \
    const int t = cell * B + ti;
#define DGMG_TILE_WW(B, LY) (whole_wave_cells<B>() && (LY) != LY_MF)
#define DGMG_TILE_THREAD(T, B) DGMG_TILE_THREAD_M(T, B, false, false)

// y = A va; optional partial of dot(w, y).
template <typename T, int B, int LY>
__global__ __launch_bounds__(kWG) void k_apply(LevelArgs<T> L, const T* __restrict__ va,
                                               T* __restrict__ y,
                                               const T* __restrict__ w, double* __restrict__ partial) {
    DGMG_TILE_THREAD_M(T, B, LY == LY_TILE, DGMG_TILE_WW(B, LY))
    double contrib = 0.0;
    const T a = row_apply<T, B, false, LY>(L, tile, lc, cell, ri, ti, active, va, nullptr);
    if (active) {
        y[t] = a;
        if (w) contrib = (double)w[t] * (double)a;
    }
    if (partial) wg_sum_store(contrib, partial);
}

// Residual r = rhs - A (va + vb), with optional epilogues: d = dinv * r * c1
// (with bj: d = c1 D_K^-1 r per cell, the cell-block Jacobi term),
// xout = va + vb, partial of ||r||^2, and restriction partials
// rp[cell, j] = sum_i P_cell(i, j) r[cell, i] (P in tile-interleaved layout)
// for the coarse correction.  r may be null when only rp is wanted.
template <typename T, int B, bool VB, int LY, bool BJ = false>
__global__ __launch_bounds__(kWG) void k_residual(LevelArgs<T> L, const T* __restrict__ va,
                                                  const T* __restrict__ vb, const T* __restrict__ rhs,
                                                  T* __restrict__ r, T* __restrict__ d, T c1,
                                                  T* __restrict__ xout, double* __restrict__ partial,
                                                  const T* __restrict__ P, T* __restrict__ rp,
                                                  const int32_t* __restrict__ ptype,
                                                  const T* __restrict__ bj) {
    DGMG_TILE_THREAD_M(T, B, LY == LY_TILE, DGMG_TILE_WW(B, LY))
    double contrib = 0.0;
    T rr = 0;
    T* lds_free = nullptr;
    const T a = row_apply<T, B, VB, LY>(L, tile, lc, cell, ri, ti, active, va, vb, &lds_free);
    if (active) rr = rhs[t] - a;
    // the block term stages the workgroup's residuals in LDS (uniform branch)
    T zb = 0;
    if constexpr (BJ) {
        if (d) zb = block_jacobi_row<T, B, LY>(bj, rr, lc, cell, ri, ti, active, lds_free);
    }
    if (active) {
        if (r) r[t] = rr;
        if (d) d[t] = BJ ? c1 * zb : L.dinv[t] * rr * c1;
        if (xout) xout[t] = VB ? va[t] + vb[t] : va[t];
        contrib = (double)rr * (double)rr;
    }
    if (P) {
        // the matrix-free product hands back a free LDS region (its own
        // occupancy is LDS-bound); the block layouts use their own
        __shared__ T rs_own[LY == LY_MF ? 1 : kWG];
        T* rs = LY == LY_MF ? lds_free : rs_own;
        if (ri < Tile<T, B>::TR) rs[ri] = rr;
        __syncthreads();
        if (active) {
            // thread (lc, j): column j of P_cell, contiguous in i (tile
            // layout, at the cell's own tile position) or strided by B
            // (row-major block of the cell's type)
            constexpr int TC = Tile<T, B>::TC, TR = Tile<T, B>::TR;
            const int j = ti;
            const int ht = cell / TC, hl = cell - ht * TC;
            const T* Pc = ptype ? P + (size_t)ptype[cell] * B * B + j : P + ((size_t)ht * B + j) * TR + hl * B;
            const int ks = ptype ? B : 1;
            const T* rc = rs + lc * B;
            T s = 0;
#pragma unroll
            for (int k = 0; k < B; ++k) s += Pc[k * ks] * rc[k];
            rp[t] = s;
        }
    }
    if (partial) wg_sum_store(contrib, partial);
}

// One inner Chebyshev step (gather vector d):
//   x += d (x = d when assign), r -= A d, dn = cd * d + cr * dinv * r
// (with bj: cr * D_K^-1 r per cell, the cell-block Jacobi term).
// On the last step of a sweep (last != 0) the sweep's final correction is
// applied at once: x = (x + d) + dn, and r, dn are not stored (the next
// sweep starts from the true residual).
template <typename T, int B, int LY, bool BJ = false>
__global__ __launch_bounds__(kWG) void k_cheb_step(LevelArgs<T> L, const T* __restrict__ d,
                                                   T* __restrict__ x, T* __restrict__ r,
                                                   T* __restrict__ dn, T cd, T cr, int assign,
                                                   int last, const T* __restrict__ bj) {
    DGMG_TILE_THREAD_M(T, B, LY == LY_TILE, DGMG_TILE_WW(B, LY))
    T* lds_free = nullptr;
    // FP32: the row's own operands are requested before the product, so that
    // their loads overlap its memory chain (FP64 keeps its register count;
    // for 3D Q1 blocks the three registers would cost a wave per SIMD)
    constexpr bool EARLY = sizeof(T) == 4 && B != 8;
    T r0 = 0, x0 = 0, di = 0;
    if (EARLY && active) {
        r0 = r[t];
        if (!assign) x0 = x[t];
        if constexpr (!BJ) di = L.dinv[t];
    }
    const T a = row_apply<T, B, false, LY>(L, tile, lc, cell, ri, ti, active, d, nullptr,
                                           BJ ? &lds_free : nullptr);
    T rr = 0;
    if (active) rr = (EARLY ? r0 : r[t]) - a;
    // the block term stages the workgroup's residuals in LDS (all threads)
    T zb = 0;
    if constexpr (BJ) zb = block_jacobi_row<T, B, LY>(bj, rr, lc, cell, ri, ti, active, lds_free);
    if (!active) return;
    const T dt = d[t];
    const T x1 = assign ? dt : (EARLY ? x0 : x[t]) + dt;
    const T dnew = cd * dt + cr * (BJ ? zb : (EARLY ? di : L.dinv[t]) * rr);
    if (last) {
        x[t] = x1 + dnew;
    } else {
        x[t] = x1;
        r[t] = rr;
        dn[t] = dnew;
    }
}

// Cell-block Jacobi (section 6 smoother with the cells' diagonal blocks as
// D): y = alpha y + beta D_K^-1 v_K at row (K, i), D_K^-1 symmetric and
// row-major per cell, so the lanes of a cell read consecutive words of
// column j; alpha = 0 does not read y.  With x given also x += y (the last
// Chebyshev step of a sweep); with vcopy given also vcopy = v (the first
// sweep from x = 0: r = b, d = c1 D^-1 b in one pass).
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_block_jacobi(int32_t n, const T* __restrict__ Dinv,
                                                      const T* __restrict__ v, T* __restrict__ y, T alpha,
                                                      T beta, T* __restrict__ x, T* __restrict__ vcopy) {
    constexpr int TC = Tile<T, B>::TC;
    const int lc = threadIdx.x / B;
    const int cell = blockIdx.x * TC + lc;
    if (lc >= TC || cell >= n) return;
    const int i = threadIdx.x - lc * B;
    const size_t t = (size_t)cell * B + i;
    const T* Dc = Dinv + (size_t)cell * B * B + i;
    const T* vc = v + (size_t)cell * B;
    T z = 0;
#pragma unroll
    for (int j = 0; j < B; ++j) z += Dc[(size_t)j * B] * vc[j];
    const T yn = alpha == T(0) ? beta * z : alpha * y[t] + beta * z;
    y[t] = yn;
    if (x) x[t] += yn;
    if (vcopy) vcopy[t] = vc[i];
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
// Restriction, second half: rc[K, j] = sum over children e of rp[e, j]
// (child ids of a group are loaded before their values).  With r given it
// also starts the coarse level's first smoothing sweep from x = 0:
// r = rc, d = cj dinv rc (point Jacobi, cj = 1 / theta of that level).
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_restrict_sum(int32_t nC, const int32_t* __restrict__ cptr,
                                                      const int32_t* __restrict__ clist,
                                                      const T* __restrict__ rp, T* __restrict__ rc,
                                                      const T* __restrict__ dinv, T* __restrict__ r,
                                                      T* __restrict__ d, T cj) {
    constexpr int G = 8;
    const int t = blockIdx.x * kWG + threadIdx.x;
    const int K = t / B, j = t - K * B;
    if (K >= nC) return;
    T acc = 0;
    const int c0 = cptr[K], c1 = cptr[K + 1];
    for (int c = c0; c < c1; c += G) {
        int e[G];
        T v[G];
#pragma unroll
        for (int q = 0; q < G; ++q) e[q] = clist[min(c + q, c1 - 1)];
#pragma unroll
        for (int q = 0; q < G; ++q) v[q] = rp[(size_t)e[q] * B + j];
#pragma unroll
        for (int q = 0; q < G; ++q)
            if (c + q < c1) acc += v[q];
    }
    rc[t] = acc;
    if (r) {
        r[t] = acc;
        d[t] = dinv[t] * acc * cj;
    }
}

// Prolongation with correction: x[e, i] += sum_j P_e(i, j) (xc + dc)[parent(e), j]
// (P tile-interleaved: one slot per tile).
template <typename T, int B>
__global__ __launch_bounds__(kWG) void k_prolong_add(int32_t n, const int32_t* __restrict__ parent,
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
    // row i of P_e: tile layout (stride TR) or the transposed block of e's
    // type (stride B); either way the lanes of a row read consecutive words
    const T* Pe = ptype ? P + (size_t)ptype[e] * B * B + i : P + (size_t)tile * B * TR + threadIdx.x;
    const size_t js = ptype ? B : TR;
    const T* v = xc + (size_t)K * B;
    T acc = 0;
    if (dc) {
        const T* w = dc + (size_t)K * B;
#pragma unroll
        for (int j = 0; j < B; ++j) acc += Pe[j * js] * (v[j] + w[j]);
    } else {
#pragma unroll
        for (int j = 0; j < B; ++j) acc += Pe[j * js] * v[j];
    }
    x[t] += acc;
}

// ------------------------------------------------------------ coarse
// x = Ainv r with the dense symmetric coarse inverse (row-major, computed in
// FP64; TA = float for the FP32 V-cycle, which reads it rounded to FP32):
// each wave owns one row and reads it with coalesced loads, accumulating in
// FP64; r is staged in LDS chunk by chunk (converted to FP64) and shared by
// the workgroup's 4 waves.
constexpr int kCoarseChunk = 4096;
template <typename Tin, typename Tout, typename TA>
__global__ __launch_bounds__(kWG) void k_coarse_solve(int32_t n, const TA* __restrict__ Ainv,
                                                      const Tin* __restrict__ r,
                                                      Tout* __restrict__ x) {
    __shared__ double rs[kCoarseChunk];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kWG / 64) + wave;
    // U independent partial sums per lane keep U loads (32 bytes) in flight;
    // column c goes to sum (c / 64) % U (chunks are multiples of 64 U)
    constexpr int U = sizeof(TA) == 4 ? 8 : 4;
    static_assert(kCoarseChunk % (64 * U) == 0, "chunk is not a multiple of a wave's sweep");
    double s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = 0.0;
    for (int c0 = 0; c0 < n; c0 += kCoarseChunk) {
        const int len = min(kCoarseChunk, n - c0);
        __syncthreads();
        for (int k = threadIdx.x; k < len; k += kWG) rs[k] = (double)r[c0 + k];
        __syncthreads();
        if (row < n) {
            const TA* a = Ainv + (size_t)row * n + c0;
            int c = lane;
            for (; c + 64 * (U - 1) < len; c += 64 * U) {
#pragma unroll
                for (int u = 0; u < U; ++u) s[u] += (double)a[c + 64 * u] * rs[c + 64 * u];
            }
#pragma unroll
            for (int u = 0; u < U - 1; ++u)
                if (c + 64 * u < len) s[u] += (double)a[c + 64 * u] * rs[c + 64 * u];
        }
    }
    double v = U == 8 ? ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]))
                      : (s[0] + s[1]) + (s[2] + s[3]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0 && row < n) x[row] = (Tout)v;
}

// ------------------------------------------------------------ vectors
template <typename T>
__global__ __launch_bounds__(kWG) void k_fill(int64_t N, T* __restrict__ x, T v) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (t < N) x[t] = v;
}

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
// With mirror (mapped pinned host memory) the 8 slots are also written there
// for the host's stopping test, instead of a separate device-to-host copy.
__global__ __launch_bounds__(kWG) void k_finalize(int32_t np, const double* __restrict__ partial,
                                                  double* __restrict__ sc, int slot, int mode,
                                                  double* __restrict__ mirror = nullptr) {
    __shared__ double red[kWG];
    // eight independent running sums keep eight loads in flight per thread
    constexpr int U = 8;
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = 0.0;
    int k = threadIdx.x;
    for (; k + (U - 1) * kWG < np; k += U * kWG) {
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] += partial[k + u * kWG];
    }
    for (; k < np; k += kWG) a[0] += partial[k];
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) s += a[u];
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
        if (mirror) {
#pragma unroll
            for (int k = 0; k < 8; ++k) mirror[k] = sc[k];
            __threadfence_system();
        }
    }
}

// x += alpha p; r -= alpha q with alpha = sc[1] / sc[2]; partial ||r||^2.
// The next V-cycle's level 0 in its precision T: when rb is set it receives
// the new residual (the right-hand side in mixed precision; in FP64 the
// V-cycle reads r itself), and when r0 is set the first smoothing sweep from
// x = 0 starts here: r0 = r, d0 = c1 dinv0 r (point Jacobi).
template <typename T>
__global__ __launch_bounds__(kWG) void k_update_xr(int64_t N, const double* __restrict__ sc,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ partial, T* __restrict__ rb,
                                                   T* __restrict__ r0, T* __restrict__ d0,
                                                   const T* __restrict__ dinv0, T c1) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const double alpha = sc[1] / sc[2];
    double v = 0.0;
    if (t < N) {
        x[t] += alpha * p[t];
        const double rn = r[t] - alpha * q[t];
        r[t] = rn;
        const T rt = (T)rn;
        if (rb) rb[t] = rt;
        if (r0) {
            r0[t] = rt;
            d0[t] = dinv0[t] * rt * c1;
        }
        v = rn * rn;
    }
    wg_sum_store(v, partial);
}

// z = a (+ b) in FP64 (the V-cycle's result) with the partials of (r, z).
template <typename Tin>
__global__ __launch_bounds__(kWG) void k_cast_dot(int64_t N, const Tin* __restrict__ a,
                                                  const Tin* __restrict__ b, double* __restrict__ z,
                                                  const double* __restrict__ r, double* __restrict__ partial) {
    const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double v = 0.0;
    if (t < N) {
        const double zz = b ? (double)a[t] + (double)b[t] : (double)a[t];
        z[t] = zz;
        v = r[t] * zz;
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
