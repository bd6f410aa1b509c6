// Matrix-free fine-level operator for meshes of identical axis-aligned boxes
// (section 3: cell and interior-face terms of a_h and the mass term of eq.
// fully_discrete, evaluated by sum factorisation instead of stored blocks).
//
// On a box of extents h the Q_p basis is a tensor product of 1D Lagrange
// polynomials on Gauss-Lobatto nodes, the Gauss-Legendre rule with p+1 points
// integrates every cell and face term exactly, and the only per-cell data is
// the (scaled) conductivity D_K.  One workgroup holds a tile of TC = 256/B
// cells (thread = one DoF row, as in the block layouts) and proceeds in
// phases separated by barriers, every cell sum factorised into 1D passes:
//   0. stage the cell's values and its 2d face neighbours' values in LDS;
//   1. u and its reference gradient at the cell quadrature points by d
//      passes of 1D contractions (x, y, z), then cM w u and the weighted
//      fluxes D grad u per point;
//   2a. per face node: the traces of both sides (the Lobatto end layers) and
//      their normal derivatives;
//   2. per face quadrature point, from the face-node data: values, conormal
//      derivatives and the face fluxes
//        f_val = (-s/2 (w_K + w_N) + sigma (u_K - u_N)) w,
//        f_con = -s/2 (u_K - u_N) w   (tested against n.D_K grad v),
//      with s = +1 when the neighbour is on the cell's upper side;
//   2b. per face and tangential node pair, the face fluxes integrated
//      against the tangential factors of the test functions;
//   3. the cell terms tested against every basis function by d passes of
//      1D contractions (z, y, x), plus the face terms times each test
//      function's normal factor.
// In phases 2a, 2 and 2b a thread takes one (axis, face node or point) pair
// and both faces normal to that axis, so the pair's index arithmetic, table
// rows and conductivity products are formed once for the two faces.
// Included by solver.hip after kernels.hpp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dgmg {

template <int B>
constexpr int mf_q() {
    return B == 4 ? 2 : B == 9 ? 3 : B == 16 ? 4 : B == 25 ? 5 : B == 8 ? 2 : B == 27 ? 3 : 4;
}
template <int D>
constexpr int npack() {
    return D * (D + 1) / 2;
}
// packed symmetric index of (a, b): 2D (xx, xy, yy); 3D (xx, xy, xz, yy, yz, zz)
template <int D>
__device__ __forceinline__ int pk(int a, int b) {
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    if constexpr (D == 2) return a == 0 ? b : 2;
    else return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

// LDS arena of the matrix-free product.  Barriers split the product into
// intervals (3D: 0 stage, 1 = 1x/2a, 2 = 1y/2, 3 = 1z/2b, 4 = 3z, 5 = 3y,
// 6 = 3x; 2D: 0 stage, 1 = 1x/2a, 2 = 1y/2, 3 = 2b/3y, 4 = 3x).  An array
// lives from the interval that writes it to the last that reads it, and
// arrays whose lives meet must not overlap; otherwise they share words, so
// the arena is as large as the largest live set (intervals 1-2):
//   xs  cell values            xn  neighbour values    (stage - 1x/2a)
//   A1  1x sums                fn  face-node data      (1x/2a - 1y/2)
//   A2  3D 1y sums             ff  face fluxes         (1y/2 - 1z/2b)
//   fq  cell terms                                     (3D 1z - 3z; 2D 1y - 3y)
//   fT  tangential integrals                           (2b - 3x)
//   A3  3D 3z sums             A4  3y sums             (3z - 3y; 3y - 3x)
//   fr  a region the caller may use once the product returns (3x on)
template <int B>
struct MfLayout {
    static constexpr int TC = kWG / B, D = dim_of<B>(), Q = mf_q<B>(), NF = 2 * D;
    static constexpr int QN = D == 3 ? Q * Q : Q;
    static constexpr int S_xs = TC * B, S_xn = TC * NF * B, S_A1 = TC * 2 * B;
    static constexpr int S_fn = TC * NF * QN * 4, S_ff = TC * NF * QN * 2, S_fT = S_ff;
    static constexpr int S_A2 = D == 3 ? TC * 3 * B : 0, S_A3 = S_A2, S_fq = TC * B * (D + 1);
    static constexpr int S_A4 = TC * 2 * B, S_fr = kWG;
    static constexpr int O_fn = 0, O_A1 = S_fn, O_xs = O_A1 + S_A1, O_xn = O_xs + S_xs;
    static constexpr int O_ff = O_xs, O_A2 = O_ff + S_ff;
    static constexpr int O_fT = 0, O_fq = D == 3 ? S_fT : O_ff + S_ff;
    static constexpr int O_A3 = O_xs, O_A4 = S_fT, O_fr = O_xs;
    static constexpr int E = D == 3 ? 6 : 4;          // the 3x interval
    struct Slot {
        int off, size, first, last;
    };
    static constexpr int NS = 11;
    static constexpr Slot slot(int k) {
        const Slot s[NS] = {{O_xs, S_xs, 0, 1},     {O_xn, S_xn, 0, 1},     {O_A1, S_A1, 1, 2},
                            {O_fn, S_fn, 1, 2},     {O_A2, S_A2, 2, 3},     {O_ff, S_ff, 2, 3},
                            {O_fq, S_fq, D == 3 ? 3 : 2, D == 3 ? 4 : 3},   {O_fT, S_fT, 3, E},
                            {O_A3, S_A3, 4, 5},     {O_A4, S_A4, D == 3 ? 5 : 3, E},
                            {O_fr, S_fr, E, E + 1}};
        return s[k];
    }
    static constexpr int size() {
        int n = 0;
        for (int k = 0; k < NS; ++k) n = slot(k).off + slot(k).size > n ? slot(k).off + slot(k).size : n;
        return n;
    }
    static constexpr bool disjoint() {
        for (int a = 0; a < NS; ++a)
            for (int b = a + 1; b < NS; ++b) {
                const Slot x = slot(a), y = slot(b);
                if (x.size == 0 || y.size == 0) continue;
                const bool live = x.first <= y.last && y.first <= x.last;
                const bool mem = x.off < y.off + y.size && y.off < x.off + x.size;
                if (live && mem) return false;
            }
        return true;
    }
};

// (A (va + vb)) at the thread's row; every thread of the workgroup must call
// it (it synchronises), `active` marks threads that own a real row.  Every
// pass below maps item i of a cell to thread i of that cell (B items).
template <typename T, int B, bool VB>
__device__ __forceinline__ T mf_row_apply(const LevelArgs<T>& L, int lc, int cell, bool active,
                                          const T* __restrict__ va, const T* __restrict__ vb,
                                          T** lds_free) {
    const MfConst<T>& C = L.mf;
    constexpr int TC = Tile<T, B>::TC, D = dim_of<B>(), Q = mf_q<B>(), NF = 2 * D;
    constexpr int QN = D == 3 ? Q * Q : Q;            // face nodes = face quadrature points
    constexpr int NP = npack<D>();
    // the 1D tables and per-axis constants, read with lane-dependent indices
    constexpr int OI = 0, OD = Q * Q, OE = 2 * Q * Q, OW = OE + 2 * Q, OH = OW + Q, OA = OH + 3, OT = OA + 3;
    __shared__ T tb[OT + 3];
    __shared__ T Dk[TC][NP];
    __shared__ T Dn[TC][NF][D];                       // row a of the neighbour's D
    __shared__ int hasn[TC][NF];                      // face has a neighbour
    using Ly = MfLayout<B>;
    static_assert(Ly::disjoint(), "arrays live in one interval overlap in the LDS arena");
    __shared__ T ar[Ly::size()];
    T(*xs)[B] = reinterpret_cast<T(*)[B]>(ar + Ly::O_xs);
    T(*xn)[NF][B] = reinterpret_cast<T(*)[NF][B]>(ar + Ly::O_xn);
    T(*ff)[NF][QN][2] = reinterpret_cast<T(*)[NF][QN][2]>(ar + Ly::O_ff);
    T(*A3)[3][B] = reinterpret_cast<T(*)[3][B]>(ar + Ly::O_A3);
    T(*fn)[NF][QN][4] = reinterpret_cast<T(*)[NF][QN][4]>(ar + Ly::O_fn);
    T(*fT)[NF][QN][2] = reinterpret_cast<T(*)[NF][QN][2]>(ar + Ly::O_fT);
    T(*A1)[2][B] = reinterpret_cast<T(*)[2][B]>(ar + Ly::O_A1);
    T(*A4)[2][B] = reinterpret_cast<T(*)[2][B]>(ar + Ly::O_A4);
    T(*A2)[3][B] = reinterpret_cast<T(*)[3][B]>(ar + Ly::O_A2);
    T(*fq)[B][D + 1] = reinterpret_cast<T(*)[B][D + 1]>(ar + Ly::O_fq);
    const T* Ig = tb + OI;
    const T* Dg = tb + OD;
    const T* Ed = tb + OE;
    const T* gw = tb + OW;
    const T* hinv = tb + OH;
    const T* area = tb + OA;
    const T* etaa = tb + OT;
    {
        const int t = threadIdx.x;
        if (t < Q * Q) {
            tb[OI + t] = C.Ig[t];
            tb[OD + t] = C.Dg[t];
        }
        if (t < 2 * Q) tb[OE + t] = C.Ed[t];
        if (t < Q) tb[OW + t] = C.gw[t];
        if (t < 3) {
            tb[OH + t] = C.hinv[t];
            tb[OA + t] = C.area[t];
            tb[OT + t] = C.eta[t];
        }
    }
    const int i = threadIdx.x - lc * B;
    const bool slot = lc < TC;                        // thread maps to a (possibly padded) cell slot
    // item coordinates of this thread (x fastest)
    const int c0 = i % Q, c1 = (i / Q) % Q, c2 = D == 3 ? i / (Q * Q) : 0;
    // face items of this thread: it = i + r B (r < FR) of the D QN pairs
    // (axis a, face node or point m), each for both faces normal to a
    constexpr int FR = (D * QN + B - 1) / B;
    int fa[FR];
#pragma unroll
    for (int r = 0; r < FR; ++r) fa[r] = (i + r * B) / QN;
    // FP32 unrolls the outer face-point loops; FP64 keeps them rolled to hold
    // its register count, and with it the occupancy
    constexpr int UF = sizeof(T) == 4 ? (D == 3 ? Q : 1) : 1;
    // ---- phase 0: stage values.  Branch-free, so that all loads of a round
    //      are in flight together: the neighbour indices, then every value
    //      and conductivity (padded slots and missing neighbours read the
    //      tile's first cell or their own, and the value is discarded).
    if (slot) {
        const int cs = active ? cell : 0;
        int nb[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int a = f >> 1;
            const int v = (f & 1) ? L.up[(size_t)a * L.n + cs] : L.lo[(size_t)a * L.n + cs];
            nb[f] = (!active || ((f & 1) && v == cs)) ? -1 : v;
        }
        auto val = [&](int c) -> T {
            return VB ? va[(size_t)c * B + i] + vb[(size_t)c * B + i] : va[(size_t)c * B + i];
        };
        const T xv = val(cs);
        const T dk = C.D[(size_t)cs * NP + (i < NP ? i : 0)];
        T wv[NF], dv[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int src = nb[f] >= 0 ? nb[f] : cs;
            wv[f] = val(src);
            dv[f] = C.D[(size_t)src * NP + pk<D>(f >> 1, i < D ? i : 0)];
        }
        xs[lc][i] = active ? xv : T(0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const bool h = nb[f] >= 0;
            xn[lc][f][i] = h ? wv[f] : T(0);
            if (i == 0) hasn[lc][f] = h;
            if (i < D) Dn[lc][f][i] = h ? dv[f] : T(0);
        }
        if (i < NP) Dk[lc][i] = active ? dk : T(0);
    }
    __syncthreads();
    // ---- phase 1x: contract x: item (g0, j1, j2) -> sum_j0 l_j0(g0) x, l_j0'(g0) x
    // ---- phase 2a: face node m of face f: traces of both sides (the Lobatto
    //      end layers) and normal derivatives sum_ja l_ja'(e) x
    if (slot) {
        T a0 = 0, b0 = 0;
#pragma unroll
        for (int j0 = 0; j0 < Q; ++j0) {
            const T x = xs[lc][j0 + Q * (c1 + Q * c2)];
            a0 += Ig[c0 * Q + j0] * x;
            b0 += Dg[c0 * Q + j0] * x;
        }
        A1[lc][0][i] = a0;
        A1[lc][1][i] = b0;
#pragma unroll
        for (int r = 0; r < FR; ++r) {
            const int it = i + r * B;
            if (it >= D * QN) break;
            const int a = fa[r], m = it - a * QN;
            // strides of the normal (sa) and tangential (st1, st2) directions
            const int sa = a == 0 ? 1 : (a == 1 ? Q : Q * Q);
            const int st1 = a == 0 ? Q : 1;
            const int st2 = D == 3 ? (a == 2 ? Q : Q * Q) : 0;
            const int J0 = (m % Q) * st1 + (D == 3 ? (m / Q) * st2 : 0);
            T xk[Q];
#pragma unroll
            for (int ja = 0; ja < Q; ++ja) xk[ja] = xs[lc][J0 + ja * sa];
#pragma unroll
            for (int s = 0; s < 2; ++s) {                 // lower (0) and upper (1) face
                const int f = 2 * a + s;
                T xm[Q];
#pragma unroll
                for (int ja = 0; ja < Q; ++ja) xm[ja] = xn[lc][f][J0 + ja * sa];
                T dK = 0, dN = 0;
#pragma unroll
                for (int ja = 0; ja < Q; ++ja) {
                    dK += C.Ed[s * Q + ja] * xk[ja];
                    dN += C.Ed[(1 - s) * Q + ja] * xm[ja];
                }
                fn[lc][f][m][0] = xk[s * (Q - 1)];
                fn[lc][f][m][1] = xm[(1 - s) * (Q - 1)];
                fn[lc][f][m][2] = dK;
                fn[lc][f][m][3] = dN;
            }
        }
    }
    __syncthreads();
    // cell terms at cell point (g0, g1, g2) from u and its reference gradient
    auto cell_terms = [&](T u, const T* gr) {
        T w = C.vol * gw[c0] * gw[c1];
        if (D == 3) w *= gw[c2];
        fq[lc][i][0] = C.cM * w * u;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T sd = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) sd += Dk[lc][pk<D>(a, b)] * hinv[b] * gr[b];
            fq[lc][i][1 + a] = w * hinv[a] * sd;
        }
    };
    // ---- phase 1y: contract y: item (g0, g1, j2)
    // ---- phase 2: face points (g1, g2) of every face: values, conormal
    //      derivatives and fluxes from the face-node data
    if (slot) {
        T u0 = 0, uy = 0, ux = 0;
#pragma unroll
        for (int j1 = 0; j1 < Q; ++j1) {
            const int src = c0 + Q * (j1 + Q * c2);
            const T iy = Ig[c1 * Q + j1], dy = Dg[c1 * Q + j1];
            u0 += iy * A1[lc][0][src];
            uy += dy * A1[lc][0][src];
            ux += iy * A1[lc][1][src];
        }
        if constexpr (D == 3) {
            A2[lc][0][i] = u0;
            A2[lc][1][i] = uy;
            A2[lc][2][i] = ux;
        } else {
            const T gr[3] = {ux, uy, T(0)};
            cell_terms(u0, gr);
        }
#pragma unroll
        for (int r = 0; r < FR; ++r) {
            const int it = i + r * B;
            if (it >= D * QN) break;
            const int a = fa[r], qf = it - a * QN;
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;   // tangential directions
            const int g1 = qf % Q, g2 = D == 3 ? qf / Q : 0;
            // D_K[a][k] / h_k of the normal (ka) and tangential (k1, k2) directions
            const T ha = hinv[a], h1 = hinv[t1], h2 = D == 3 ? hinv[t2] : T(0);
            const T daa = Dk[lc][pk<D>(a, a)];
            const T ka = daa * ha, k1 = Dk[lc][pk<D>(a, t1)] * h1;
            const T k2 = D == 3 ? Dk[lc][pk<D>(a, t2)] * h2 : T(0);
            const T wq = area[a] * gw[g1] * (D == 3 ? gw[g2] : T(1));
            const T eh = etaa[a] * T(0.5);
#pragma unroll
            for (int s = 0; s < 2; ++s) {                 // s = 1: neighbour on the upper side
                const int f = 2 * a + s;
                const T sgn = s ? T(1) : T(-1);
                T uK = 0, uN = 0, nK = 0, nN = 0, p1K = 0, p1N = 0, p2K = 0, p2N = 0;
                // sums over m1 first, then weighted by the m2 factor (the
                // tensor weights are never formed)
#pragma unroll UF
                for (int m2 = 0; m2 < (D == 3 ? Q : 1); ++m2) {
                    T a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
#pragma unroll
                    for (int m1 = 0; m1 < Q; ++m1) {
                        const T* nd = fn[lc][f][m1 + Q * m2];
                        const T iy = Ig[g1 * Q + m1], dy = Dg[g1 * Q + m1];
                        a0 += iy * nd[0];
                        a1 += iy * nd[1];
                        a2 += iy * nd[2];
                        a3 += iy * nd[3];
                        a4 += dy * nd[0];
                        a5 += dy * nd[1];
                    }
                    if (D == 3) {
                        const T i2 = Ig[g2 * Q + m2], e2 = Dg[g2 * Q + m2];
                        uK += i2 * a0;
                        uN += i2 * a1;
                        nK += i2 * a2;
                        nN += i2 * a3;
                        p1K += i2 * a4;
                        p1N += i2 * a5;
                        p2K += e2 * a0;
                        p2N += e2 * a1;
                    } else {
                        uK = a0;
                        uN = a1;
                        nK = a2;
                        nN = a3;
                        p1K = a4;
                        p1N = a5;
                    }
                }
                const T* dn = Dn[lc][f];
                T wK = ka * nK + k1 * p1K;
                T wN = dn[a] * ha * nN + dn[t1] * h1 * p1N;
                if (D == 3) {
                    wK += k2 * p2K;
                    wN += dn[t2] * h2 * p2N;
                }
                const T w = hasn[lc][f] ? wq : T(0);      // boundary face: no terms
                const T sig = eh * (daa + dn[a]);
                const T jmp = uK - uN;
                // value flux, and the conormal flux factor: it is tested against
                // n.D_K grad v, i.e. times D_K[a][k] / h_k for each direction k
                ff[lc][f][qf][0] = (T(-0.5) * sgn * (wK + wN) + sig * jmp) * w;
                ff[lc][f][qf][1] = T(-0.5) * sgn * jmp * w;
            }
        }
    }
    __syncthreads();
    // ---- phase 1z (3D): contract z, cell terms at point (g0, g1, g2)
    // ---- phase 2b: per face and tangential node pair m = (m1, m2), the face
    //      fluxes integrated against the tangential factors of the test
    //      functions: fT[.][0] = sum_q (f_val tI + f_con_t1 t1' + f_con_t2 t2'),
    //      fT[.][1] = sum_q f_con_a tI; a test function then needs only its
    //      normal factor
    // ---- (2D) phase 3y: contract the cell terms over g1: items (g0, i1)
    if (slot) {
        if constexpr (D == 3) {
            T u = 0, gr[3] = {0, 0, 0};
#pragma unroll
            for (int j2 = 0; j2 < Q; ++j2) {
                const int src = c0 + Q * (c1 + Q * j2);
                const T iz = Ig[c2 * Q + j2], dz = Dg[c2 * Q + j2];
                u += iz * A2[lc][0][src];
                gr[1] += iz * A2[lc][1][src];
                gr[0] += iz * A2[lc][2][src];
                gr[2] += dz * A2[lc][0][src];
            }
            cell_terms(u, gr);
        } else {
            T P = 0, X = 0;
#pragma unroll
            for (int g1 = 0; g1 < Q; ++g1) {
                const T* F = fq[lc][c0 + Q * g1];
                const T iy = Ig[g1 * Q + c1], dy = Dg[g1 * Q + c1];
                P += iy * F[0] + dy * F[2];
                X += iy * F[1];
            }
            A4[lc][0][i] = P;
            A4[lc][1][i] = X;
        }
#pragma unroll
        for (int r = 0; r < FR; ++r) {
            const int it = i + r * B;
            if (it >= D * QN) break;
            const int a = fa[r], m = it - a * QN;
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const int m1 = m % Q, m2 = D == 3 ? m / Q : 0;
            // D_K[a][k] / h_k of the normal (ka) and tangential (k1, k2) directions
            const T ka = Dk[lc][pk<D>(a, a)] * hinv[a];
            const T k1 = Dk[lc][pk<D>(a, t1)] * hinv[t1];
            const T k2 = D == 3 ? Dk[lc][pk<D>(a, t2)] * hinv[t2] : T(0);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int f = 2 * a + s;
                T sv = 0, sc = 0;
                // sums over g1 first, then weighted by the g2 factor
#pragma unroll UF
                for (int g2 = 0; g2 < (D == 3 ? Q : 1); ++g2) {
                    T e0 = 0, e1 = 0;
#pragma unroll
                    for (int g1 = 0; g1 < Q; ++g1) {
                        const T* F = ff[lc][f][g1 + Q * g2];
                        const T i1 = Ig[g1 * Q + m1], d1 = Dg[g1 * Q + m1];
                        e0 += F[0] * i1 + k1 * F[1] * d1;
                        e1 += F[1] * i1;
                    }
                    if (D == 3) {
                        const T i2 = Ig[g2 * Q + m2], d2 = Dg[g2 * Q + m2];
                        sv += i2 * e0 + k2 * e1 * d2;
                        sc += i2 * e1;
                    } else {
                        sv = e0;
                        sc = e1;
                    }
                }
                fT[lc][f][m][0] = sv;
                fT[lc][f][m][1] = ka * sc;
            }
        }
    }
    __syncthreads();
    if constexpr (D == 3) {
        // ---- phase 3z: items (g0, g1, i2): W = sum_g2 (l_i2(g2) c0 + l_i2'(g2) c3),
        //      X = sum_g2 l_i2(g2) c1, Y = sum_g2 l_i2(g2) c2 of the cell terms c
        if (slot) {
            T W = 0, X = 0, Y = 0;
#pragma unroll
            for (int g2 = 0; g2 < Q; ++g2) {
                const T* F = fq[lc][c0 + Q * (c1 + Q * g2)];
                const T iz = Ig[g2 * Q + c2], dz = Dg[g2 * Q + c2];
                W += iz * F[0] + dz * F[3];
                X += iz * F[1];
                Y += iz * F[2];
            }
            A3[lc][0][i] = W;
            A3[lc][1][i] = X;
            A3[lc][2][i] = Y;
        }
        __syncthreads();
        // ---- phase 3y: items (g0, i1, i2): P = sum_g1 (l_i1(g1) W + l_i1'(g1) Y),
        //      X' = sum_g1 l_i1(g1) X
        if (slot) {
            T P = 0, X = 0;
#pragma unroll
            for (int g1 = 0; g1 < Q; ++g1) {
                const int src = c0 + Q * (g1 + Q * c2);
                const T iy = Ig[g1 * Q + c1], dy = Dg[g1 * Q + c1];
                P += iy * A3[lc][0][src] + dy * A3[lc][2][src];
                X += iy * A3[lc][1][src];
            }
            A4[lc][0][i] = P;
            A4[lc][1][i] = X;
        }
        __syncthreads();
    }
    // ---- phase 3x: test function I = (i0, i1, i2): sum_g0 (l_i0(g0) P + l_i0'(g0) X'),
    //      plus the face terms times the test function's normal factor.
    if (lds_free) *lds_free = ar + Ly::O_fr;
    T y = 0;
    if (slot) {
#pragma unroll
        for (int g0 = 0; g0 < Q; ++g0) {
            const int src = g0 + Q * (c1 + Q * c2);
            y += Ig[g0 * Q + c0] * A4[lc][0][src] + Dg[g0 * Q + c0] * A4[lc][1][src];
        }
        const int ik[3] = {c0, c1, c2};
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int a = f >> 1, eK = f & 1;
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const int m = ik[t1] + (D == 3 ? Q * ik[t2] : 0);
            // normal factor: trace (0 or 1 at the Lobatto ends) and derivative
            if (ik[a] == eK * (Q - 1)) y += fT[lc][f][m][0];
            y += Ed[eK * Q + ik[a]] * fT[lc][f][m][1];
        }
    }
    return y;
}

}  // namespace dgmg
