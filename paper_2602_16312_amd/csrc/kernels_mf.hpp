// Matrix-free fine-level operator for meshes of identical axis-aligned boxes
// (section 3: cell and interior-face terms of a_h and the mass term of eq.
// fully_discrete, evaluated by sum factorisation instead of stored blocks).
//
// On a box of extents h the Q_p basis is a tensor product of 1D Lagrange
// polynomials on Gauss-Lobatto nodes, the Gauss-Legendre rule with p+1 points
// integrates every cell and face term exactly, and the only per-cell data is
// the (scaled) conductivity D_K.  One workgroup holds a tile of TC = 256/B
// cells (thread = one DoF row, as in the block layouts) and proceeds in
// phases separated by barriers:
//   0. stage the cell's values and its 2d face neighbours' values in LDS;
//   1. thread g evaluates u and grad u at cell quadrature point g and stores
//      cM w u and the weighted fluxes D grad u;
//   2. threads evaluate, at the face quadrature points, the traces and
//      conormal derivatives of both sides and store the face fluxes
//        f_val = (-s/2 (w_K + w_N) + sigma (u_K - u_N)) w,
//        f_con = -s/2 (u_K - u_N) w   (tested against n.D_K grad v),
//      with s = +1 when the neighbour is on the cell's upper side;
//   2b. per face and tangential node pair, the face fluxes are integrated
//      against the tangential factors of the test functions;
//   3. thread I integrates the cell terms against its basis function and
//      adds the face terms times its normal factor.
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

// (A (va + vb)) at the thread's row; every thread of the workgroup must call
// it (it synchronises), `active` marks threads that own a real row.
template <typename T, int B, bool VB>
__device__ __forceinline__ T mf_row_apply(const LevelArgs<T>& L, int lc, int cell, bool active,
                                          const T* __restrict__ va, const T* __restrict__ vb) {
    const MfConst<T>& C = L.mf;
    constexpr int TC = Tile<T, B>::TC, D = dim_of<B>(), Q = mf_q<B>(), NF = 2 * D;
    constexpr int QF = D == 3 ? Q * Q : Q;            // face quadrature points
    constexpr int NP = npack<D>();
    __shared__ T xs[TC][B];
    __shared__ T xn[TC][NF][B];
    __shared__ T Dk[TC][NP];
    __shared__ T Dn[TC][NF][D];                       // row a of the neighbour's D
    __shared__ T fq[TC][B][D + 1];
    __shared__ T ff[TC][NF][QF][D + 1];
    __shared__ T fT[TC][NF][QF][2];                   // face fluxes integrated tangentially
    __shared__ int hasn[TC][NF];                      // face has a neighbour
    const int i = threadIdx.x - lc * B;
    const bool slot = lc < TC;                        // thread maps to a (possibly padded) cell slot
    // ---- phase 0: stage values
    if (slot) {
        T v = 0;
        if (active) v = VB ? va[(size_t)cell * B + i] + vb[(size_t)cell * B + i] : va[(size_t)cell * B + i];
        xs[lc][i] = v;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int a = f >> 1;
            int nb = -1;
            if (active) {
                nb = (f & 1) ? L.up[(size_t)a * L.n + cell] : L.lo[(size_t)a * L.n + cell];
                if ((f & 1) && nb == cell) nb = -1;
            }
            T w = 0;
            if (nb >= 0) w = VB ? va[(size_t)nb * B + i] + vb[(size_t)nb * B + i] : va[(size_t)nb * B + i];
            xn[lc][f][i] = w;
            if (i == 0) hasn[lc][f] = nb >= 0;
            if (i < D) {
                Dn[lc][f][i] = nb >= 0 ? C.D[(size_t)nb * NP + pk<D>(a, i)] : T(0);
            }
        }
        if (i < NP) Dk[lc][i] = active ? C.D[(size_t)cell * NP + i] : T(0);
    }
    __syncthreads();
    // ---- phase 1: cell quadrature point g = i
    if (slot) {
        int gk[3] = {i % Q, (i / Q) % Q, D == 3 ? i / (Q * Q) : 0};
        T u = 0, gr[3] = {0, 0, 0};
        if constexpr (D == 2) {
            for (int j1 = 0; j1 < Q; ++j1) {
                T sI = 0, sD = 0;
#pragma unroll
                for (int j0 = 0; j0 < Q; ++j0) {
                    const T x = xs[lc][j0 + Q * j1];
                    sI += C.Ig[gk[0] * Q + j0] * x;
                    sD += C.Dg[gk[0] * Q + j0] * x;
                }
                const T a1 = C.Ig[gk[1] * Q + j1], d1 = C.Dg[gk[1] * Q + j1];
                u += a1 * sI;
                gr[0] += a1 * sD;
                gr[1] += d1 * sI;
            }
        } else {
            for (int j2 = 0; j2 < Q; ++j2) {
                const T a2 = C.Ig[gk[2] * Q + j2], d2 = C.Dg[gk[2] * Q + j2];
                for (int j1 = 0; j1 < Q; ++j1) {
                    T sI = 0, sD = 0;
#pragma unroll
                    for (int j0 = 0; j0 < Q; ++j0) {
                        const T x = xs[lc][j0 + Q * (j1 + Q * j2)];
                        sI += C.Ig[gk[0] * Q + j0] * x;
                        sD += C.Dg[gk[0] * Q + j0] * x;
                    }
                    const T a1 = C.Ig[gk[1] * Q + j1], d1 = C.Dg[gk[1] * Q + j1];
                    u += a1 * a2 * sI;
                    gr[0] += a1 * a2 * sD;
                    gr[1] += d1 * a2 * sI;
                    gr[2] += a1 * d2 * sI;
                }
            }
        }
        T w = C.vol;
#pragma unroll
        for (int k = 0; k < D; ++k) w *= C.gw[gk[k]];
        fq[lc][i][0] = C.cM * w * u;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T s = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) s += Dk[lc][pk<D>(a, b)] * C.hinv[b] * gr[b];
            fq[lc][i][1 + a] = w * C.hinv[a] * s;
        }
    }
    // ---- phase 2: face quadrature points (runtime face index: strides instead
    // of indexed register arrays)
    if (slot) {
        for (int it = i; it < NF * QF; it += B) {
            const int f = it / QF, qf = it - f * QF;
            const int a = f >> 1;
            const int side = f & 1;                  // 1: neighbour on the upper side
            const T s = side ? T(1) : T(-1);
            const int eK = side, eN = 1 - side;      // face at xi_a = eK of K, xi_a = eN of N
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;   // tangential directions
            const int sa = a == 0 ? 1 : (a == 1 ? Q : Q * Q);
            const int s1 = t1 == 0 ? 1 : Q;
            const int s2 = D == 3 ? (t2 == 1 ? Q : Q * Q) : 0;
            const int g1 = qf % Q, g2 = D == 3 ? qf / Q : 0;
            // Lobatto nodes contain both ends, so a trace is the face layer of
            // nodes (layer 0 or Q-1); the normal derivative needs every layer
            const int lK = eK * (Q - 1), lN = eN * (Q - 1);
            T uK = 0, uN = 0, nK = 0, nN = 0, p1K = 0, p1N = 0, p2K = 0, p2N = 0;
            for (int j2 = 0; j2 < (D == 3 ? Q : 1); ++j2) {
                const T i2 = D == 3 ? C.Ig[g2 * Q + j2] : T(1);
                const T e2 = D == 3 ? C.Dg[g2 * Q + j2] : T(0);
                for (int j1 = 0; j1 < Q; ++j1) {
                    const T tI = C.Ig[g1 * Q + j1] * i2;
                    const T t1d = C.Dg[g1 * Q + j1] * i2;
                    const T t2d = C.Ig[g1 * Q + j1] * e2;
                    const int J0 = j1 * s1 + j2 * s2;
                    T dnK = 0, dnN = 0;
#pragma unroll
                    for (int ja = 0; ja < Q; ++ja) {
                        dnK += C.Ed[eK * Q + ja] * xs[lc][J0 + ja * sa];
                        dnN += C.Ed[eN * Q + ja] * xn[lc][f][J0 + ja * sa];
                    }
                    const T vK = xs[lc][J0 + lK * sa], vN = xn[lc][f][J0 + lN * sa];
                    uK += tI * vK;
                    uN += tI * vN;
                    nK += tI * dnK;
                    nN += tI * dnN;
                    p1K += t1d * vK;
                    p1N += t1d * vN;
                    p2K += t2d * vK;
                    p2N += t2d * vN;
                }
            }
            T wK = Dk[lc][pk<D>(a, a)] * C.hinv[a] * nK + Dk[lc][pk<D>(a, t1)] * C.hinv[t1] * p1K;
            T wN = Dn[lc][f][a] * C.hinv[a] * nN + Dn[lc][f][t1] * C.hinv[t1] * p1N;
            if (D == 3) {
                wK += Dk[lc][pk<D>(a, t2)] * C.hinv[t2] * p2K;
                wN += Dn[lc][f][t2] * C.hinv[t2] * p2N;
            }
            T w = C.area[a] * C.gw[g1] * (D == 3 ? C.gw[g2] : T(1));
            if (!hasn[lc][f]) w = 0;                  // boundary face: no terms
            const T sig = C.eta[a] * T(0.5) * (Dk[lc][pk<D>(a, a)] + Dn[lc][f][a]);
            const T jmp = uK - uN;
            ff[lc][f][qf][0] = (T(-0.5) * s * (wK + wN) + sig * jmp) * w;
            const T fc = T(-0.5) * s * jmp * w;
            ff[lc][f][qf][1 + a] = fc * Dk[lc][pk<D>(a, a)] * C.hinv[a];
            ff[lc][f][qf][1 + t1] = fc * Dk[lc][pk<D>(a, t1)] * C.hinv[t1];
            if (D == 3) ff[lc][f][qf][1 + t2] = fc * Dk[lc][pk<D>(a, t2)] * C.hinv[t2];
        }
    }
    __syncthreads();
    // ---- phase 2b: per face and tangential node pair m = (m1, m2), the face
    // fluxes integrated against the tangential factors of the test functions:
    // fT[.][0] = sum_q (f_val tI + f_con_t1 t1' + f_con_t2 t2'), fT[.][1] =
    // sum_q f_con_a tI; a test function then needs only its normal factor
    if (slot) {
        for (int it = i; it < NF * QF; it += B) {
            const int f = it / QF, m = it - f * QF;
            const int a = f >> 1;
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const int m1 = m % Q, m2 = D == 3 ? m / Q : 0;
            T sv = 0, sn = 0;
            for (int qf = 0; qf < QF; ++qf) {
                const int g1 = qf % Q, g2 = D == 3 ? qf / Q : 0;
                const T i1 = C.Ig[g1 * Q + m1], i2 = D == 3 ? C.Ig[g2 * Q + m2] : T(1);
                const T* F = ff[lc][f][qf];
                sv += F[0] * i1 * i2 + F[1 + t1] * C.Dg[g1 * Q + m1] * i2;
                if (D == 3) sv += F[1 + t2] * i1 * C.Dg[g2 * Q + m2];
                sn += F[1 + a] * i1 * i2;
            }
            fT[lc][f][m][0] = sv;
            fT[lc][f][m][1] = sn;
        }
    }
    __syncthreads();
    // ---- phase 3: test against the thread's basis function I = i (direct
    // sums; with the loops unrolled the compiler keeps the 1D table entries
    // in registers, which measured faster than factorising the sums)
    T y = 0;
    if (slot) {
        const int ik[3] = {i % Q, (i / Q) % Q, D == 3 ? i / (Q * Q) : 0};
        for (int g = 0; g < B; ++g) {
            const int gk[3] = {g % Q, (g / Q) % Q, D == 3 ? g / (Q * Q) : 0};
            T pI[3], pD[3];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                pI[k] = C.Ig[gk[k] * Q + ik[k]];
                pD[k] = C.Dg[gk[k] * Q + ik[k]];
            }
            T val = pI[0];
#pragma unroll
            for (int k = 1; k < D; ++k) val *= pI[k];
            y += fq[lc][g][0] * val;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                T dv = pD[a];
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k != a) dv *= pI[k];
                y += fq[lc][g][1 + a] * dv;
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int a = f >> 1, eK = f & 1;
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const int m = ik[t1] + (D == 3 ? Q * ik[t2] : 0);
            // normal factor: trace (0 or 1 at the Lobatto ends) and derivative
            if (ik[a] == eK * (Q - 1)) y += fT[lc][f][m][0];
            y += C.Ed[eK * Q + ik[a]] * fT[lc][f][m][1];
        }
    }
    return y;
}

}  // namespace dgmg
