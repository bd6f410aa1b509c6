// Kernels of the discrete adjoint of the semi-implicit step (reverse mode of
// section 3.1's step map with respect to per-cell conductivity scalings).
//
// A(s) = sum_K s_K G_K (every term of a_h carries one conductivity tensor and
// the penalty averages the two sides' n^T D n), so the conductivity gradient
// of a term lambda^T A(s) U is  lambda^T G_K U  per cell: the cell stiffness
// part plus, on every face of K, the face matrix of K's side alone.
// All reductions are deterministic (fixed order, no atomics).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ionic.hpp"

namespace dgmg {

// d/du of the gate coefficients and of I_ion (FHN and Aliev-Panfilov).
__device__ __forceinline__ void ionic_derivs(const IonicParams& P, double u, const double* w,
                                             double* dIu, double* dIw, double* dc1, double* dc0) {
    const double* p = P.p;
    const double k = p[0], a = p[1];
    const double cubic = k * (3.0 * u * u - 2.0 * (a + 1.0) * u + a);
    if (P.model == 0) {
        *dIu = cubic;
        dIw[0] = 1.0;
        dc1[0] = 0.0;
        dc0[0] = p[2];
    } else {
        *dIu = cubic + w[0];
        dIw[0] = u;
        dc1[0] = 0.0;
        dc0[0] = -p[2] * k * (2.0 * u - a - 1.0);
    }
}

// Reverse of (gate update, ionic current, load vector) of one step, given
// lambda = A_0^-1 Ubar_{n+1} and the incoming adjoint of W_{n+1}:
//   fbar = M lambda, gbar = -chi fbar, Wtot = Wbar_{n+1} + dI/dw gbar,
//   Ustar_bar = dI/du gbar + sum_s Wtot * dt_eff (c0' + W_{n+1} c1') / den,
// accumulated into Ubar_n, Ubar_{n-1}, Wbar_n, Wbar_{n-1}.  W_{n+1} is
// recomputed from (W_n, W_{n-1}) exactly as in the forward step.
// Workgroups hold whole cells (blockDim = B * cells).
template <int B>
__global__ __launch_bounds__(256) void k_adjoint_step(int32_t n, IonicParams P, double cU,
                                                      const double* __restrict__ mass,
                                                      const double* __restrict__ U,
                                                      const double* __restrict__ Up,
                                                      const double* __restrict__ W,
                                                      const double* __restrict__ Wp,
                                                      const double* __restrict__ lam,
                                                      const double* __restrict__ Wbar_in,
                                                      double* __restrict__ Ubar,
                                                      double* __restrict__ Upbar,
                                                      double* __restrict__ Wbar,
                                                      double* __restrict__ Wpbar) {
    const int cells_per = blockDim.x / B;
    const int lc = threadIdx.x / B, i = threadIdx.x - lc * B;
    const int cell = blockIdx.x * cells_per + lc;
    if (lc >= cells_per || cell >= n) return;
    const int64_t N = (int64_t)n * B;
    const int64_t t = (int64_t)cell * B + i;
    // fbar_i = sum_j M_ij lambda_j  (cell mass block, column-major, padded stride)
    const double* M = mass + (size_t)cell * ((B * B + 1) / 2 * 2) + i;
    const double* lc_ = lam + (size_t)cell * B;
    double fb = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) fb += M[j * B] * lc_[j];
    const double gb = -P.chi * fb;
    const bool bdf2 = P.bdf == 2;
    const double us = bdf2 ? 2.0 * U[t] - Up[t] : U[t];
    const double dte = bdf2 ? 2.0 * P.dt : P.dt;
    double c1[3], c0[3], w[3], den[3];
    gate_coeffs(P, us, c1, c0);
    for (int s = 0; s < P.S; ++s) {
        den[s] = bdf2 ? 3.0 - 2.0 * P.dt * c1[s] : 1.0 - P.dt * c1[s];
        const double num = bdf2 ? 4.0 * W[s * N + t] - Wp[s * N + t] + 2.0 * P.dt * c0[s]
                                : W[s * N + t] + P.dt * c0[s];
        w[s] = num / den[s];
    }
    double dIu, dIw[3], dc1[3], dc0[3];
    ionic_derivs(P, us, w, &dIu, dIw, dc1, dc0);
    double usb = dIu * gb;
    for (int s = 0; s < P.S; ++s) {
        const double wt = Wbar_in[s * N + t] + dIw[s] * gb;
        usb += wt * dte * (dc0[s] + w[s] * dc1[s]) / den[s];
        Wbar[s * N + t] += (bdf2 ? 4.0 : 1.0) * wt / den[s];
        if (bdf2) Wpbar[s * N + t] -= wt / den[s];
    }
    if (bdf2) {
        Ubar[t] += 4.0 * cU * fb + 2.0 * usb;
        Upbar[t] -= cU * fb + usb;
    } else {
        Ubar[t] += cU * fb + usb;
    }
}

// Per face: q[2f + side] = -lambda_f^T X_side U_f over the face's 2B DoFs
// (X column-major, 2B x 2B per side).  Thread = (face in group, row I).
template <int B>
__global__ __launch_bounds__(256) void k_grad_faces(int32_t nf, const int64_t* __restrict__ fc,
                                                    const double* __restrict__ X,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ q) {
    constexpr int R = 2 * B;
    constexpr int FPW = 256 / R;
    __shared__ double sp[256], sm[256];
    const int lf = threadIdx.x / R, I = threadIdx.x - lf * R;
    const int f = blockIdx.x * FPW + lf;
    const bool active = lf < FPW && f < nf;
    double vp = 0.0, vm = 0.0;
    if (active) {
        const int64_t cp = fc[2 * (size_t)f], cm = fc[2 * (size_t)f + 1];
        const double* Xp = X + (size_t)f * 2 * R * R + I;
        const double* Xm = Xp + (size_t)R * R;
        const double* up = U + (size_t)cp * B;
        const double* um = U + (size_t)cm * B;
        double ap = 0.0, am = 0.0;
#pragma unroll
        for (int J = 0; J < B; ++J) {
            ap += Xp[J * R] * up[J];
            am += Xm[J * R] * up[J];
        }
#pragma unroll
        for (int J = 0; J < B; ++J) {
            ap += Xp[(B + J) * R] * um[J];
            am += Xm[(B + J) * R] * um[J];
        }
        const double l = I < B ? lam[(size_t)cp * B + I] : lam[(size_t)cm * B + (I - B)];
        vp = l * ap;
        vm = l * am;
    }
    sp[threadIdx.x] = vp;
    sm[threadIdx.x] = vm;
    __syncthreads();
    if (active && I == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < R; ++k) {
            a += sp[threadIdx.x + k];
            b += sm[threadIdx.x + k];
        }
        q[2 * (size_t)f] = -a;
        q[2 * (size_t)f + 1] = -b;
    }
}

// Per cell: grad[K] += -lambda_K^T S_K U_K + sum over K's faces of q[face, K's side].
template <int B>
__global__ __launch_bounds__(256) void k_grad_cells(int32_t n, const double* __restrict__ S,
                                                    const int32_t* __restrict__ nptr,
                                                    const int32_t* __restrict__ ncode,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ grad) {
    __shared__ double sv[256];
    const int cells_per = 256 / B;
    const int lc = threadIdx.x / B, i = threadIdx.x - lc * B;
    const int cell = blockIdx.x * cells_per + lc;
    const bool active = lc < cells_per && cell < n;
    double v = 0.0;
    if (active) {
        const double* Sc = S + (size_t)cell * B * B + i;   // column-major (i, j) at j*B + i
        const double* uc = U + (size_t)cell * B;
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < B; ++j) a += Sc[j * B] * uc[j];
        v = lam[(size_t)cell * B + i] * a;
    }
    sv[threadIdx.x] = v;
    __syncthreads();
    if (active && i == 0) {
        double a = 0.0;
        for (int k = 0; k < B; ++k) a += sv[threadIdx.x + k];
        double g = -a;
        for (int e = nptr[cell]; e < nptr[cell + 1]; ++e) {
            const int code = ncode[e];
            g += q[2 * (size_t)(code >> 1) + (code & 1)];
        }
        grad[cell] += g;
    }
}

// Sensor misfit at one time: r_k = sum_i w_{k,i} U[cell_k, i] - target_k;
// loss[0] += sum_k r_k^2 and, when Ubar is set, Ubar += sum_k 2 r_k e_k.
// One workgroup; sensors in chunks of 256, scatter serialised per DoF index
// so that sensors sharing a cell never race.
template <int B>
__global__ __launch_bounds__(256) void k_sensor_misfit(int32_t ns, const int64_t* __restrict__ scell,
                                                       const double* __restrict__ sw,
                                                       const double* __restrict__ U,
                                                       const double* __restrict__ target,
                                                       double* __restrict__ Ubar,
                                                       double* __restrict__ loss) {
    __shared__ double r[256];
    double lsum = 0.0;
    for (int k0 = 0; k0 < ns; k0 += 256) {
        const int k = k0 + threadIdx.x;
        double rk = 0.0;
        if (k < ns) {
            const double* u = U + (size_t)scell[k] * B;
            for (int i = 0; i < B; ++i) rk += sw[(size_t)k * B + i] * u[i];
            rk -= target[k];
        }
        r[threadIdx.x] = rk;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int kk = 0; kk < min(256, ns - k0); ++kk) lsum += r[kk] * r[kk];
        if (Ubar && (int)threadIdx.x < B)
            for (int kk = 0; kk < min(256, ns - k0); ++kk)
                Ubar[(size_t)scell[k0 + kk] * B + threadIdx.x] +=
                    2.0 * r[kk] * sw[(size_t)(k0 + kk) * B + threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] += lsum;
}

}  // namespace dgmg
