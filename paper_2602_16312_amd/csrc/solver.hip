// Device solver: level upload, V-cycle, PCG, time step and the C ABI.
//
// V-cycle (section 6: one V-cycle per PCG iteration, Chebyshev-accelerated
// Jacobi of degree k with s pre- and post-smoothing sweeps; section 5.1:
// prolongation by the natural embedding, restriction by its transpose,
// Galerkin level operators): on level l < L-1
//   x = Cheb(b, 0); r = b - A x; e = V(P^T r); x += P e; x = Cheb(b, x)
// and the coarsest level is solved exactly with the FP64 inverse of its
// Cholesky-factorised operator.  Chebyshev (Saad's preconditioned Chebyshev
// acceleration, D = diag(A_l)) restarts s times from the true residual; the
// sweep's last step also applies its final "x += d" (for degree 1 that
// correction is carried as pending and fused into the next kernel that
// reads x).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <type_traits>
#include <vector>

#include "adjoint.hpp"
#include "internal.hpp"
#include "ionic.hpp"
#include "kernels.hpp"
#include "kernels_multi.hpp"
#include "kernels_mf.hpp"

namespace dgmg {

static thread_local std::string g_last_error;
void set_last_error(const std::string& m) { g_last_error = m; }
[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            fail(DGMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

// level layout: LYV (LY_TILE, LY_AXIS, LY_MF, LY_AXS) and AXV (axis-ELL) as constants
#define DISPATCH_LY(lyval, ...)                                                        \
    switch (lyval) {                                                                   \
        case LY_TILE: { constexpr int LYV = LY_TILE; constexpr bool AXV = false; __VA_ARGS__; } break; \
        case LY_AXIS: { constexpr int LYV = LY_AXIS; constexpr bool AXV = true; __VA_ARGS__; } break;  \
        case LY_AXS: { constexpr int LYV = LY_AXS; constexpr bool AXV = true; __VA_ARGS__; } break;    \
        default: { constexpr int LYV = LY_MF; constexpr bool AXV = false; __VA_ARGS__; } break;        \
    }

#define DISPATCH_B(bval, ...)                                                          \
    switch (bval) {                                                                    \
        case 4: { constexpr int BV = 4; __VA_ARGS__; } break;                          \
        case 8: { constexpr int BV = 8; __VA_ARGS__; } break;                          \
        case 9: { constexpr int BV = 9; __VA_ARGS__; } break;                          \
        case 16: { constexpr int BV = 16; __VA_ARGS__; } break;                        \
        case 25: { constexpr int BV = 25; __VA_ARGS__; } break;                        \
        case 27: { constexpr int BV = 27; __VA_ARGS__; } break;                        \
        case 64: { constexpr int BV = 64; __VA_ARGS__; } break;                        \
        default: fail(DGMG_EUNSUPPORTED, "unsupported block size");                    \
    }

void* DeviceMemory::alloc(size_t bytes) const {
    void* p = nullptr;
    if (has_user) {
        p = user.alloc(user.ctx, bytes);
        if (!p) fail(DGMG_ENOMEM, "the caller's allocator returned NULL");
        if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
            user.free(user.ctx, p);
            fail(DGMG_EINVAL, "the caller's allocator returned memory that is not 256-byte aligned");
        }
        return p;
    }
    if (hipMalloc(&p, bytes) != hipSuccess) fail(DGMG_ENOMEM, "hipMalloc failed");
    return p;
}

void DeviceMemory::release(void* p) const noexcept {
    if (!p) return;
    if (has_user)
        user.free(user.ctx, p);
    else
        (void)hipFree(p);
}

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static inline unsigned blocks_for(int64_t threads) { return (unsigned)((threads + kWG - 1) / kWG); }

// coarse problems above this size are factorised on the device at set-up
constexpr int64_t kHostCholeskyMax = 4096;

struct DevLevel {
    int32_t n = 0, nf = 0;
    int64_t N = 0;
    int32_t *slot_ptr = nullptr, *snb = nullptr;          // tile-ELL structure
    bool ax = false;                                       // axis-ELL layout instead
    bool sf = false;                                       // axis-ELL with sparse face blocks
    bool mf = false;                                       // matrix-free boxes (fine level)
    MfConst<double> mf64{};
    MfConst<float> mf32{};
    int32_t *up = nullptr, *lo = nullptr;                  // axis-ELL neighbours
    int32_t *child_ptr = nullptr, *child_list = nullptr;  // children on level l-1
    int32_t* parent = nullptr;                             // parent on level l+1
    int32_t* ptype = nullptr;                              // P_e = table[ptype[e]] when set
    int32_t* cmap = nullptr;                               // tile-ELL: tile position -> cell
    int32_t ntypes = 0;                                    // distinct blocks in that table
    double *vals64 = nullptr, *dinv64 = nullptr, *P64 = nullptr;
    float *vals32 = nullptr, *dinv32 = nullptr, *P32 = nullptr;
    double* bj64 = nullptr;                                // cell-block Jacobi: D_K^-1 (symmetric)
    float* bj32 = nullptr;
    void *vb = nullptr, *vx = nullptr, *vx2 = nullptr, *vr = nullptr, *vd = nullptr, *vd2 = nullptr;
    double lam_lo = 0, lam_hi = 0;
};

}  // namespace dgmg

using namespace dgmg;

struct dgmg_hierarchy : public Hierarchy {};

struct dgmg_solver {
    int dim = 0, p = 0, b = 0, L = 0, prec = 0, S = 1, bdf = 2;
    int cheb_k = 3, cheb_s = 3;
    int max_rhs = 1, mfma = 0;
    int fine_layout = 0;              // DGMG_LAYOUT_*
    int jacobi = 0;                   // DGMG_JACOBI_*
    std::vector<std::vector<double>> bjinv;   // cell-block Jacobi: D_K^-1 per smoothed level
    // matrix-free fine level on identical boxes: extents, packed scaled D,
    // mass coefficient and penalty factors per axis
    double mf_h[3] = {0, 0, 0};
    double mf_cM = 0.0, mf_eta[3] = {0, 0, 0};
    std::vector<double> mf_D;
    std::vector<int> axis0;           // axis of every fine face (face order of ops[0])
    // levels >= 1 whose agglomerates form a conforming grid of boxes: axis of
    // every face and whether its stored (plus, minus) order runs downwards
    std::vector<std::vector<int>> axisl;
    std::vector<std::vector<char>> flipl;
    int64_t N = 0;
    bool on_device = false;
    std::vector<DevLevel> lv;
    // coarse
    int64_t nc_dofs = 0;
    double* Ainv = nullptr;     // dense coarse inverse (FP64 solvers)
    float* Ainv32 = nullptr;    // the same rounded to FP32 (mixed solvers' FP32 V-cycle)
    // outer PCG work
    double *r = nullptr, *z = nullptr, *zold = nullptr, *pv = nullptr, *q = nullptr, *bwork = nullptr;
    double *tmp64a = nullptr, *tmp64b = nullptr;
    double* partial = nullptr;
    double* sc = nullptr;
    double* sc_host = nullptr;
    double* sc_host_dev = nullptr;   // device address of the pinned sc_host (mapped)
    double* scratch = nullptr;     // this device's static PCG scratch (dgmg_pcg_solve_noalloc)
    int32_t* act = nullptr;        // per-column active mask of multi-column PCG
    int32_t* act_host = nullptr;   // pinned staging of that mask
    double* mass = nullptr;
    // adjoint data (optional)
    bool has_adjoint = false;
    double *adjS = nullptr, *adjX = nullptr, *adjq = nullptr;
    int64_t* adj_fc = nullptr;
    int32_t *adj_nptr = nullptr, *adj_ncode = nullptr;
    int64_t nf0 = 0;
    // sensors (optional)
    int32_t n_sensors = 0;
    int64_t* scell = nullptr;
    double* sw = nullptr;
    IonicParams ip{};
    double cU = 0.0;
    std::vector<void*> allocs;
    int64_t dev_bytes = 0;
    // host copies
    std::vector<BlockOp> ops;
    std::vector<std::vector<double>> Ph;
    std::vector<std::vector<int64_t>> parents;
    std::vector<double> mass_h;
    dgmg_solver_info info{};
    // roctx ranges (time step, PCG solve, V-cycle level) for rocprofv3's
    // marker trace: on when DGMG_ROCTX=1 at set-up
    bool roctx = false;
    // per-phase events of the time step (ionic, load vector, PCG), created
    // when phase timing is first switched on; phase_n: steps timed since
    int phase_on = 0, phase_n = 0;
    hipEvent_t phase_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // kernel timing with HIP events (one kernel kind on one level at a time)
    int prof_kind = -1, prof_level = -1;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
    size_t prof_used = 0;

    DeviceMemory mem;
    template <typename T>
    T* dalloc(size_t count) {
        if (count == 0) count = 1;
        void* p = mem.alloc(count * sizeof(T));
        allocs.push_back(p);
        dev_bytes += (int64_t)(count * sizeof(T));
        return (T*)p;
    }
    // releases a dalloc'ed block of `bytes` before the solver ends
    void dfree(void* p, size_t bytes) {
        for (size_t k = 0; k < allocs.size(); ++k)
            if (allocs[k] == p) {
                allocs.erase(allocs.begin() + (ptrdiff_t)k);
                mem.release(p);
                dev_bytes -= (int64_t)bytes;
                return;
            }
    }
    template <typename T>
    T* upload(const std::vector<T>& h) {
        T* d = dalloc<T>(h.size());
        HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }
    ~dgmg_solver() {
        for (hipEvent_t e : phase_ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : prof_ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        for (void* p : allocs) mem.release(p);
        if (sc_host) (void)hipHostFree(sc_host);
        if (act_host) (void)hipHostFree(act_host);
    }
};

namespace dgmg {

// padded block stride of the device layout (whole 16-byte vectors)
template <typename T>
static size_t block_stride(int b) {
    const size_t ev = 16 / sizeof(T);
    return ((size_t)b * b + ev - 1) / ev * ev;
}

// row-major b x b blocks -> column-major with padded stride, converted to T
template <typename T>
static std::vector<T> to_colmajor(const std::vector<double>& a, int b) {
    const size_t bb = (size_t)b * b, nblk = a.size() / bb, bs = block_stride<T>(b);
    std::vector<T> out(nblk * bs, (T)0);
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < nblk; ++k)
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) out[k * bs + (size_t)j * b + i] = (T)a[k * bb + (size_t)i * b + j];
    return out;
}

template <typename T>
static LevelArgs<T> largs(const DevLevel& L);
template <>
LevelArgs<double> largs<double>(const DevLevel& L) {
    return {L.vals64, L.slot_ptr, L.snb, L.dinv64, L.n, L.up, L.lo, L.mf64, L.cmap};
}
template <>
LevelArgs<float> largs<float>(const DevLevel& L) {
    return {L.vals32, L.slot_ptr, L.snb, L.dinv32, L.n, L.up, L.lo, L.mf32, L.cmap};
}
static int level_ly(const DevLevel& L) { return L.mf ? LY_MF : (L.ax ? (L.sf ? LY_AXS : LY_AXIS) : LY_TILE); }
template <typename T>
static const T* Pof(const DevLevel& L);
template <>
const double* Pof<double>(const DevLevel& L) { return L.P64; }
template <>
const float* Pof<float>(const DevLevel& L) { return L.P32; }
template <typename T>
static const T* BJof(const DevLevel& L);
template <>
const double* BJof<double>(const DevLevel& L) { return L.bj64; }
template <>
const float* BJof<float>(const DevLevel& L) { return L.bj32; }
// the prolongation's blocks: with a type table, its transposed half
template <typename T>
static const T* PofT(const DevLevel& L, int b) {
    return Pof<T>(L) + (L.ptype ? (size_t)L.ntypes * b * b : 0);
}

// Selects the event pair of one launch when that kernel kind/level is being
// timed (see dgmg_profile_begin); klaunch attaches the pair to the launch.
struct ProfScope {
    dgmg_solver* s;
    bool on = false;
    size_t idx = 0;
    ProfScope(dgmg_solver* s_, int kind, int level, hipStream_t) : s(s_) {
        if (s->prof_kind != kind || s->prof_level != level) return;
        if (s->prof_used == s->prof_ev.size()) {
            hipEvent_t a, b;
            HIPCHK(hipEventCreate(&a));
            HIPCHK(hipEventCreate(&b));
            s->prof_ev.push_back({a, b});
        }
        idx = s->prof_used++;
        on = true;
    }
};

// Launches kernel k on st.  When the scope is timing this launch, the start
// and stop events ride on the kernel's own dispatch (hipExtLaunchKernelGGL),
// so their interval is the kernel's execution alone, without the dispatch
// gaps that separately recorded events would add.
template <typename... KA, typename... A>
static void klaunch(const ProfScope& ps, void (*k)(KA...), dim3 grid, dim3 block, hipStream_t st,
                    A&&... a) {
    if (!ps.on) {
        hipLaunchKernelGGL(k, grid, block, 0, st, static_cast<KA>(a)...);
        return;
    }
    hipExtLaunchKernelGGL(k, grid, block, 0, st, ps.s->prof_ev[ps.idx].first, ps.s->prof_ev[ps.idx].second, 0,
                          static_cast<KA>(a)...);
}
enum { PK_CHEB_STEP = 0, PK_RESIDUAL = 1, PK_APPLY = 2, PK_RESTRICT = 3, PK_PROLONG = 4,
       PK_COARSE = 5 };

static int level_index(const dgmg_solver* s, const DevLevel& L) { return (int)(&L - s->lv.data()); }

// ---------------------------------------------------------------- launchers
template <typename T, int B>
static unsigned tiles_for(const DevLevel& L) {
    return (unsigned)((L.n + Tile<T, B>::TC - 1) / Tile<T, B>::TC);
}
// number of workgroups (tiles) of the block kernels on a level; also the
// number of partial sums they write
template <typename T>
static unsigned level_tiles(const dgmg_solver* s, const DevLevel& L) {
    unsigned g = 0;
    DISPATCH_B(s->b, g = tiles_for<T, BV>(L));
    return g;
}
template <typename T, int R = 1>
static void launch_apply(dgmg_solver* s, const DevLevel& L, const T* va, T* y, const T* w,
                         double* partial, hipStream_t st) {
    ProfScope ps(s, PK_APPLY, level_index(s, L), st);
    DISPATCH_LY(level_ly(L), {
        if constexpr (R == 1) {
            DISPATCH_B(s->b, klaunch(ps, k_apply<T, BV, LYV>, tiles_for<T, BV>(L), kWG, st, largs<T>(L), va, y, w,
                                                                                        partial));
        } else if constexpr (LYV == LY_AXS) {
            fail(DGMG_EUNSUPPORTED, "sparse face blocks have no multi-column kernels");
        } else if constexpr (LYV == LY_MF) {
            fail(DGMG_EUNSUPPORTED, "the matrix-free fine level has no multi-column kernels");
        } else {
            DISPATCH_B(s->b, klaunch(ps, k_apply_m<T, BV, R, AXV>, tiles_for<T, BV>(L), kWG, st, largs<T>(L), va, y,
                                                                                            w, partial));
        }
    });
}
template <typename T, int R = 1>
static void launch_residual(dgmg_solver* s, const DevLevel& L, const T* va, const T* vb, const T* rhs,
                            T* r, T* d, T c1, T* xout, double* partial, hipStream_t st,
                            const T* P = nullptr, T* rp = nullptr, const int32_t* ptype = nullptr,
                            const T* bj = nullptr) {
    ProfScope ps(s, PK_RESIDUAL, level_index(s, L), st);
    if (R != 1 && bj) fail(DGMG_EUNSUPPORTED, "cell-block Jacobi is single-column only");
    DISPATCH_LY(level_ly(L), {
        if constexpr (R == 1) {
            if (vb && bj) {
                DISPATCH_B(s->b, klaunch(ps, k_residual<T, BV, true, LYV, true>, tiles_for<T, BV>(L), kWG, st,
                                     largs<T>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype, bj));
            } else if (vb) {
                DISPATCH_B(s->b, klaunch(ps, k_residual<T, BV, true, LYV>, tiles_for<T, BV>(L), kWG, st,
                                     largs<T>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype, bj));
            } else if (bj) {
                DISPATCH_B(s->b, klaunch(ps, k_residual<T, BV, false, LYV, true>, tiles_for<T, BV>(L), kWG, st,
                                     largs<T>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype, bj));
            } else {
                DISPATCH_B(s->b, klaunch(ps, k_residual<T, BV, false, LYV>, tiles_for<T, BV>(L), kWG, st,
                                     largs<T>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype, bj));
            }
        } else if constexpr (LYV == LY_AXS) {
            fail(DGMG_EUNSUPPORTED, "sparse face blocks have no multi-column kernels");
        } else if constexpr (LYV == LY_MF) {
            fail(DGMG_EUNSUPPORTED, "the matrix-free fine level has no multi-column kernels");
        } else {
            bool done = false;
            if constexpr (std::is_same<T, float>::value && R == 8) {
                if (s->mfma && s->b == 8) {
                    if (((uintptr_t)va | (uintptr_t)vb) & 15)
                        fail(DGMG_EINVAL, "8-column vectors must be 16-byte aligned");
                    if (vb)
                        klaunch(ps, k_residual_m<float, 8, 8, true, AXV, true>, tiles_for<float, 8>(L), kWG, st,
                            largs<float>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype);
                    else
                        klaunch(ps, k_residual_m<float, 8, 8, false, AXV, true>, tiles_for<float, 8>(L), kWG, st,
                            largs<float>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype);
                    done = true;
                }
            }
            if (!done) {
                if (vb) {
                    DISPATCH_B(s->b, klaunch(ps, k_residual_m<T, BV, R, true, AXV>, tiles_for<T, BV>(L), kWG, st,
                                         largs<T>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype));
                } else {
                    DISPATCH_B(s->b, klaunch(ps, k_residual_m<T, BV, R, false, AXV>, tiles_for<T, BV>(L), kWG, st,
                                         largs<T>(L), va, vb, rhs, r, d, c1, xout, partial, P, rp, ptype));
                }
            }
        }
    });
}
template <typename T, int R = 1>
static void launch_step(dgmg_solver* s, const DevLevel& L, const T* d, T* x, T* r, T* dn, T cd, T cr,
                        int assign, int last, hipStream_t st, const T* bj = nullptr) {
    ProfScope ps(s, PK_CHEB_STEP, level_index(s, L), st);
    if (R != 1 && bj) fail(DGMG_EUNSUPPORTED, "cell-block Jacobi is single-column only");
    DISPATCH_LY(level_ly(L), {
        if constexpr (R == 1) {
            if (bj) {
                DISPATCH_B(s->b, klaunch(ps, k_cheb_step<T, BV, LYV, true>, tiles_for<T, BV>(L), kWG, st,
                                         largs<T>(L), d, x, r, dn, cd, cr, assign, last, bj));
            } else {
                DISPATCH_B(s->b, klaunch(ps, k_cheb_step<T, BV, LYV>, tiles_for<T, BV>(L), kWG, st, largs<T>(L), d,
                                         x, r, dn, cd, cr, assign, last, bj));
            }
        } else if constexpr (LYV == LY_AXS) {
            fail(DGMG_EUNSUPPORTED, "sparse face blocks have no multi-column kernels");
        } else if constexpr (LYV == LY_MF) {
            fail(DGMG_EUNSUPPORTED, "the matrix-free fine level has no multi-column kernels");
        } else {
            bool done = false;
            if constexpr (std::is_same<T, float>::value && R == 8) {
                if (s->mfma && s->b == 8) {
                    if ((uintptr_t)d & 15) fail(DGMG_EINVAL, "8-column vectors must be 16-byte aligned");
                    klaunch(ps, k_cheb_step_mfma8<AXV>, tiles_for<float, 8>(L), kWG, st, largs<float>(L), d, x, r, dn,
                                                                                  cd, cr, assign, last);
                    done = true;
                }
            }
            if (!done) {
                DISPATCH_B(s->b, klaunch(ps, k_cheb_step_m<T, BV, R, AXV>, tiles_for<T, BV>(L), kWG, st,
                                     largs<T>(L), d, x, r, dn, cd, cr, assign, last));
            }
        }
    });
}

template <typename T, int R = 1>
static void coarse_solve(dgmg_solver* s, const T* rc, T* xc, hipStream_t st) {
    const int n = (int)s->nc_dofs;
    ProfScope ps(s, PK_COARSE, s->L - 1, st);
    const int rows_per_wg = kWG / 64;   // one row per wave
    // the FP32 V-cycle of a mixed solver reads the inverse rounded to FP32
    using TA = T;
    const TA* A;
    if constexpr (sizeof(T) == 4) A = s->Ainv32;
    else A = s->Ainv;
    if (!A) fail(DGMG_EINVAL, "the coarse inverse of this precision is not held by the solver");
    if constexpr (R == 1)
        klaunch(ps, k_coarse_solve<T, T, TA>, (n + rows_per_wg - 1) / rows_per_wg, kWG, st, n, A, rc, xc);
    else
        klaunch(ps, k_coarse_solve_m<T, T, R, TA>, (n + rows_per_wg - 1) / rows_per_wg, kWG, st, n, A, rc, xc);
}

// A roctx range (host timeline of rocprofv3's marker trace) for the scope's
// lifetime when the solver has them switched on.
struct RangeScope {
    bool on;
    RangeScope(const dgmg_solver* s, const char* name) : on(s->roctx) {
        if (on) roctxRangePushA(name);
    }
    ~RangeScope() {
        if (on) roctxRangePop();
    }
};
static const char* vcycle_range_name(int l) {
    static const char* names[DGMG_MAX_LEVELS] = {"dgmg V-cycle level 0", "dgmg V-cycle level 1",
        "dgmg V-cycle level 2", "dgmg V-cycle level 3", "dgmg V-cycle level 4", "dgmg V-cycle level 5",
        "dgmg V-cycle level 6", "dgmg V-cycle level 7"};
    return l < DGMG_MAX_LEVELS ? names[l] : "dgmg V-cycle level";
}

// One V-cycle from level l on R columns; the result is x + d (d may be null).
// init_done: the producer of the level's right-hand side already started the
// first smoothing sweep from x = 0 (r = b, d = c1 dinv b in the level's r
// and d buffers), so that sweep skips its init kernel.
template <typename T, int R = 1>
static void vcycle(dgmg_solver* s, int l, hipStream_t st, T** xres, T** dres, bool init_done = false) {
    RangeScope range(s, vcycle_range_name(l));
    DevLevel& L = s->lv[l];
    T* b = (T*)L.vb;
    if (l == s->L - 1) {
        coarse_solve<T, R>(s, b, (T*)L.vx, st);
        *xres = (T*)L.vx;
        *dres = nullptr;
        return;
    }
    const int64_t NR = L.N * R;
    const double theta = 0.5 * (L.lam_hi + L.lam_lo), delta = 0.5 * (L.lam_hi - L.lam_lo);
    const double sigma1 = theta / delta;
    const T c1 = (T)(1.0 / theta);
    T *x = (T*)L.vx, *x2 = (T*)L.vx2, *r = (T*)L.vr, *d = (T*)L.vd, *d2 = (T*)L.vd2;
    bool xzero = true, pending = false;
    const T* dinv = largs<T>(L).dinv;
    // cell-block Jacobi (single column): the fused kernels apply the cells'
    // inverse diagonal blocks D_K^-1 in their epilogue instead of 1/diag
    const T* bjp = (R == 1 && s->jacobi == DGMG_JACOBI_CELL_BLOCK) ? BJof<T>(L) : nullptr;
    auto sweep = [&]() {
        if (xzero && !pending && init_done) {
            init_done = false;   // r and d were written by the right-hand side's producer
        } else if (xzero && !pending) {
            if constexpr (R == 1) {
                if (bjp) {   // r = b and d = c1 D^-1 b in one pass
                    DISPATCH_B(s->b, k_block_jacobi<T, BV><<<tiles_for<T, BV>(L), kWG, 0, st>>>(
                                         L.n, bjp, b, d, T(0), c1, (T*)nullptr, r));
                } else {
                    k_cheb_init0<T><<<blocks_for(L.N), kWG, 0, st>>>(L.N, b, dinv, r, d, c1);
                }
            } else {
                k_cheb_init0_m<T, R><<<blocks_for(NR), kWG, 0, st>>>(NR, b, dinv, r, d, c1);
            }
        } else if (pending) {
            // r = b - A(x + d), materialise x + d into x2
            launch_residual<T, R>(s, L, xzero ? d : x, xzero ? nullptr : d, b, r, d2, c1, x2, nullptr, st,
                                  nullptr, nullptr, nullptr, bjp);
            std::swap(x, x2);
            std::swap(d, d2);
            xzero = false;
        } else {
            launch_residual<T, R>(s, L, x, (const T*)nullptr, b, r, d, c1, (T*)nullptr, nullptr, st, nullptr,
                                  nullptr, nullptr, bjp);
        }
        double rho = 1.0 / sigma1;
        for (int i = 1; i < s->cheb_k; ++i) {
            const double rn = 1.0 / (2.0 * sigma1 - rho);
            // the last step of the sweep also applies the sweep's final
            // correction x += d (it needs only the row's own new d)
            const int last = i == s->cheb_k - 1;
            const T cr = (T)(2.0 * rn / delta);
            launch_step<T, R>(s, L, d, x, r, d2, (T)(rn * rho), cr, xzero ? 1 : 0, last, st, bjp);
            xzero = false;
            if (!last) std::swap(d, d2);
            rho = rn;
        }
        // degree 1: the correction from the residual kernel stays pending and
        // is applied by the next kernel that reads x
        pending = s->cheb_k == 1;
    };
    for (int k = 0; k < s->cheb_s; ++k) sweep();
    // residual for the coarse correction (materialising a pending update),
    // with the per-cell restriction partials P_e^T r_e in its epilogue
    DevLevel& C = s->lv[l + 1];
    T* rp = d2;   // free: no step result or pending correction lives there
    if (pending) {
        launch_residual<T, R>(s, L, xzero ? d : x, xzero ? nullptr : d, b, (T*)nullptr, (T*)nullptr, c1, x2,
                              nullptr, st, Pof<T>(L), rp, L.ptype);
        std::swap(x, x2);
        xzero = false;
        pending = false;
    } else {
        if (xzero) {
            // no smoothing: x = 0 and r = b
            k_fill<T><<<blocks_for(NR), kWG, 0, st>>>(NR, x, (T)0);
            xzero = false;
        }
        launch_residual<T, R>(s, L, x, (const T*)nullptr, b, (T*)nullptr, (T*)nullptr, c1, (T*)nullptr,
                              nullptr, st, Pof<T>(L), rp, L.ptype);
    }
    // the coarse level's first sweep (point Jacobi, single column) starts in
    // the restriction kernel
    const bool init_c = R == 1 && l + 1 < s->L - 1 && s->cheb_s > 0 && s->jacobi != DGMG_JACOBI_CELL_BLOCK;
    {
    ProfScope ps(s, PK_RESTRICT, l, st);
    if constexpr (R == 1) {
        const T c1c = (T)(1.0 / (0.5 * (C.lam_hi + C.lam_lo)));
        DISPATCH_B(s->b, klaunch(ps, k_restrict_sum<T, BV>, blocks_for(C.N), kWG, st, C.n, C.child_ptr, C.child_list,
                                 rp, (T*)C.vb, largs<T>(C).dinv, init_c ? (T*)C.vr : (T*)nullptr,
                                 init_c ? (T*)C.vd : (T*)nullptr, c1c));
    } else {
        DISPATCH_B(s->b, klaunch(ps, k_restrict_sum_m<T, BV, R>, blocks_for(C.N * R), kWG, st,
                             C.n, C.child_ptr, C.child_list, rp, (T*)C.vb));
    }
    }
    T *xc, *dc;
    vcycle<T, R>(s, l + 1, st, &xc, &dc, init_c);
    {
    ProfScope ps(s, PK_PROLONG, l, st);
    if constexpr (R == 1) {
        DISPATCH_B(s->b, klaunch(ps, k_prolong_add<T, BV>, tiles_for<T, BV>(L), kWG, st, L.n, L.parent, PofT<T>(L, s->b), xc,
                                                                                     dc, x, L.ptype));
    } else {
        DISPATCH_B(s->b, klaunch(ps, k_prolong_add_m<T, BV, R>, tiles_for<T, BV>(L), kWG, st, L.n, L.parent,
                                                                                         PofT<T>(L, s->b), xc, dc, x, L.ptype));
    }
    }
    for (int k = 0; k < s->cheb_s; ++k) sweep();
    // hand back the level's buffers as they are now named
    L.vx = x;
    L.vx2 = x2;
    L.vd = d;
    L.vd2 = d2;
    *xres = x;
    *dres = pending ? d : nullptr;
}

// z = V(r), r and z FP64 of length N x R (column-minor).  Single column:
// `rb_ready` says that the FP32 copy of r is already in the level-0 right-hand
// side (written by the PCG update), and a non-null `rz_partial` makes the exit
// cast also write the partials of (r, z).
template <int R = 1>
static void apply_vcycle(dgmg_solver* s, const double* r, double* z, hipStream_t st, bool rb_ready = false,
                         double* rz_partial = nullptr, bool init_done = false) {
    DevLevel& L0 = s->lv[0];
    const int64_t NR = s->N * R;
    if (s->prec == DGMG_PREC_FP64) {
        L0.vb = (void*)r;
        double *x, *d;
        vcycle<double, R>(s, 0, st, &x, &d, R == 1 && init_done);
        if (R == 1 && rz_partial)
            k_cast_dot<double><<<blocks_for(NR), kWG, 0, st>>>(NR, x, d, z, r, rz_partial);
        else
            k_cast<double, double><<<blocks_for(NR), kWG, 0, st>>>(NR, x, d, z);
    } else {
        if (!(R == 1 && rb_ready))
            k_cast<double, float><<<blocks_for(NR), kWG, 0, st>>>(NR, r, nullptr, (float*)L0.vb);
        float *x, *d;
        vcycle<float, R>(s, 0, st, &x, &d, R == 1 && init_done);
        if (R == 1 && rz_partial)
            k_cast_dot<float><<<blocks_for(NR), kWG, 0, st>>>(NR, x, d, z, r, rz_partial);
        else
            k_cast<float, double><<<blocks_for(NR), kWG, 0, st>>>(NR, x, d, z);
    }
}

static double read_scalars(dgmg_solver* s, hipStream_t st, int R = 1, const double* sc = nullptr) {
    HIPCHK(hipMemcpyAsync(s->sc_host, sc ? sc : s->sc, 8 * (size_t)R * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
    return s->sc_host[0];
}
// The last finalize kernel before this already wrote the 8 scalars into the
// mapped pinned host buffer: wait for it.
static double wait_scalars(dgmg_solver* s, hipStream_t st) {
    HIPCHK(hipStreamSynchronize(st));
    return s->sc_host[0];
}

// Names the failed CG quantity: (p, A p) <= 0 means A_0 is not positive
// definite along p; (r, z) <= 0 means the V-cycle is not.
static std::string breakdown_msg(int its, int col, double pq, double gam) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "PCG breakdown at iteration %d%s%s: (p, A p) = %.6e, (r, z) = %.6e (%s)", its,
                  col >= 0 ? " of column " : "", col >= 0 ? std::to_string(col).c_str() : "", pq, gam,
                  !(pq > 0.0) ? "operator not positive definite along p" : "preconditioner not positive definite");
    return buf;
}

// The reduction scratch (block partials and the 8 scalar slots: 0 ||r||^2,
// 1 gamma = (r, z), 2 (p, A p), 3 the new (r, z), 4 beta, 5 (r_new, z_old),
// 6 ||b||^2) is passed in: the solver's own buffers, or the static array of
// the non-allocating entry point.
static int pcg(dgmg_solver* s, const double* b, double* x, const dgmg_pcg_opts& o, dgmg_pcg_stats* stats,
               hipStream_t st, double* partial, double* sc) {
    RangeScope range(s, "dgmg PCG");
    const int64_t N = s->N;
    const unsigned nb = blocks_for(N);
    DevLevel& L0 = s->lv[0];
    const unsigned nt = level_tiles<double>(s, L0);   // partials of the block kernels
    // r = b - A x, ||r||^2
    launch_residual<double>(s, L0, x, nullptr, b, s->r, nullptr, 1.0, nullptr, partial, st);
    const bool relb = o.tol_mode == DGMG_TOL_REL_B;
    k_finalize<<<1, kWG, 0, st>>>(nt, partial, sc, 0, 0, relb ? nullptr : s->sc_host_dev);
    double bnorm = 0.0;
    if (relb) {
        k_dot<<<nb, kWG, 0, st>>>(N, b, b, partial);
        k_finalize<<<1, kWG, 0, st>>>(nb, partial, sc, 6, 0, s->sc_host_dev);
    }
    wait_scalars(s, st);
    const double r0 = std::sqrt(s->sc_host[0]);
    if (o.tol_mode == DGMG_TOL_REL_B) bnorm = std::sqrt(s->sc_host[6]);
    if (!std::isfinite(r0)) fail(DGMG_ENAN, "non-finite initial residual");
    const double thresh = o.tol_mode == DGMG_TOL_ABS ? o.tol : (o.tol_mode == DGMG_TOL_REL_B ? o.tol * bnorm : o.tol * r0);
    stats->its = 0;
    stats->r0 = r0;
    stats->rfin = r0;
    stats->converged = 0;
    if (r0 == 0.0 || r0 <= thresh) {
        stats->converged = 1;
        return DGMG_OK;
    }
    apply_vcycle(s, s->r, s->z, st);
    k_dot<<<nb, kWG, 0, st>>>(N, s->r, s->z, partial);
    k_finalize<<<1, kWG, 0, st>>>(nb, partial, sc, 1, 0);
    k_update_p<<<nb, kWG, 0, st>>>(N, sc, s->z, s->pv, 1);
    int its = 0;
    // mixed precision: the update also writes the FP32 right-hand side of the next V-cycle;
    // with point Jacobi it also starts that V-cycle's first level-0 sweep (r, d)
    float* rb = s->prec == DGMG_PREC_MIXED ? (float*)L0.vb : nullptr;
    const bool init0 = s->L > 1 && s->cheb_s > 0 && s->jacobi != DGMG_JACOBI_CELL_BLOCK;
    const double c1_0 = 1.0 / (0.5 * (L0.lam_hi + L0.lam_lo));
    while (its < o.max_it) {
        launch_apply<double>(s, L0, s->pv, s->q, s->pv, partial, st);
        k_finalize<<<1, kWG, 0, st>>>(nt, partial, sc, 2, 0);
        if (s->prec == DGMG_PREC_MIXED)
            k_update_xr<float><<<nb, kWG, 0, st>>>(N, sc, s->pv, s->q, x, s->r, partial, rb,
                                                   init0 ? (float*)L0.vr : nullptr, init0 ? (float*)L0.vd : nullptr,
                                                   L0.dinv32, (float)c1_0);
        else
            k_update_xr<double><<<nb, kWG, 0, st>>>(N, sc, s->pv, s->q, x, s->r, partial, (double*)nullptr,
                                                    init0 ? (double*)L0.vr : nullptr,
                                                    init0 ? (double*)L0.vd : nullptr, L0.dinv64, c1_0);
        k_finalize<<<1, kWG, 0, st>>>(nb, partial, sc, 0, 0, s->sc_host_dev);
        wait_scalars(s, st);
        ++its;
        const double gam = s->sc_host[1], pq = s->sc_host[2];
        const double rn = std::sqrt(s->sc_host[0]);
        stats->its = its;
        stats->rfin = rn;
        if (!(pq > 0.0) || !(gam > 0.0)) {
            if (!std::isfinite(pq) || !std::isfinite(gam)) fail(DGMG_ENAN, "non-finite PCG scalar");
            fail(DGMG_ENOTSPD, breakdown_msg(its, -1, pq, gam));
        }
        if (!std::isfinite(rn)) fail(DGMG_ENAN, "non-finite residual");
        if (rn <= thresh) {
            stats->converged = 1;
            return DGMG_OK;
        }
        if (o.flexible) {
            std::swap(s->z, s->zold);
            apply_vcycle(s, s->r, s->z, st, true, nullptr, init0);
            k_dot<<<nb, kWG, 0, st>>>(N, s->r, s->zold, partial);
            k_finalize<<<1, kWG, 0, st>>>(nb, partial, sc, 5, 0);
            k_dot<<<nb, kWG, 0, st>>>(N, s->r, s->z, partial);
        } else {
            // z = V(r) with the partials of (r, z) from the exit cast
            apply_vcycle(s, s->r, s->z, st, true, partial, init0);
        }
        k_finalize<<<1, kWG, 0, st>>>(nb, partial, sc, 3, o.flexible ? 2 : 1);
        k_update_p<<<nb, kWG, 0, st>>>(N, sc, s->z, s->pv, 0);
    }
    return DGMG_NOT_CONVERGED;
}

// PCG on R columns at once: every A_0 apply, V-cycle and reduction serves all
// columns; alpha, beta and the stopping test are per column.  A converged
// column is frozen (alpha = 0) while the others iterate.
template <int R>
static int pcg_multi(dgmg_solver* s, const double* b, double* x, const dgmg_pcg_opts& o,
                     dgmg_pcg_stats* stats, hipStream_t st) {
    const int64_t N = s->N, NR = N * R;
    const unsigned nb = blocks_for(N);
    DevLevel& L0 = s->lv[0];
    const unsigned nt = level_tiles<double>(s, L0);
    launch_residual<double, R>(s, L0, x, nullptr, b, s->r, nullptr, 1.0, nullptr, s->partial, st);
    k_finalize_m<R><<<1, kWG, 0, st>>>(nt, s->partial, s->sc, 0, 0);
    if (o.tol_mode == DGMG_TOL_REL_B) {
        k_dot_m<R><<<nb, kWG, 0, st>>>(N, b, b, s->partial);
        k_finalize_m<R><<<1, kWG, 0, st>>>(nb, s->partial, s->sc, 6, 0);
    }
    read_scalars(s, st, R);
    double thresh[R];
    int n_active = 0;
    for (int c = 0; c < R; ++c) {
        const double r0 = std::sqrt(s->sc_host[c]);
        if (!std::isfinite(r0)) fail(DGMG_ENAN, "non-finite initial residual");
        const double bn = o.tol_mode == DGMG_TOL_REL_B ? std::sqrt(s->sc_host[6 * R + c]) : 0.0;
        thresh[c] = o.tol_mode == DGMG_TOL_ABS ? o.tol : (o.tol_mode == DGMG_TOL_REL_B ? o.tol * bn : o.tol * r0);
        stats[c].its = 0;
        stats[c].r0 = r0;
        stats[c].rfin = r0;
        const bool done = r0 == 0.0 || r0 <= thresh[c];
        stats[c].converged = done ? 1 : 0;
        s->act_host[c] = done ? 0 : 1;
        n_active += done ? 0 : 1;
    }
    if (n_active == 0) return DGMG_OK;
    // the pinned mask is rewritten only after the next synchronisation of st
    HIPCHK(hipMemcpyAsync(s->act, s->act_host, R * sizeof(int32_t), hipMemcpyHostToDevice, st));
    apply_vcycle<R>(s, s->r, s->z, st);
    k_dot_m<R><<<nb, kWG, 0, st>>>(N, s->r, s->z, s->partial);
    k_finalize_m<R><<<1, kWG, 0, st>>>(nb, s->partial, s->sc, 1, 0);
    k_update_p_m<R><<<blocks_for(NR), kWG, 0, st>>>(NR, s->sc, s->z, s->pv, 1);
    int its = 0;
    while (its < o.max_it) {
        launch_apply<double, R>(s, L0, s->pv, s->q, s->pv, s->partial, st);
        k_finalize_m<R><<<1, kWG, 0, st>>>(nt, s->partial, s->sc, 2, 0);
        k_update_xr_m<R><<<nb, kWG, 0, st>>>(N, s->sc, s->act, s->pv, s->q, x, s->r, s->partial);
        k_finalize_m<R><<<1, kWG, 0, st>>>(nb, s->partial, s->sc, 0, 0);
        read_scalars(s, st, R);
        ++its;
        n_active = 0;
        for (int c = 0; c < R; ++c) {
            if (!s->act_host[c]) continue;
            const double gam = s->sc_host[1 * R + c], pq = s->sc_host[2 * R + c];
            const double rn = std::sqrt(s->sc_host[c]);
            stats[c].its = its;
            stats[c].rfin = rn;
            if (!(pq > 0.0) || !(gam > 0.0)) {
                if (!std::isfinite(pq) || !std::isfinite(gam)) fail(DGMG_ENAN, "non-finite PCG scalar");
                fail(DGMG_ENOTSPD, breakdown_msg(its, c, pq, gam));
            }
            if (!std::isfinite(rn)) fail(DGMG_ENAN, "non-finite residual");
            if (rn <= thresh[c]) {
                stats[c].converged = 1;
                s->act_host[c] = 0;
            } else {
                ++n_active;
            }
        }
        if (n_active == 0) return DGMG_OK;
        HIPCHK(hipMemcpyAsync(s->act, s->act_host, R * sizeof(int32_t), hipMemcpyHostToDevice, st));
        if (o.flexible) std::swap(s->z, s->zold);
        apply_vcycle<R>(s, s->r, s->z, st);
        if (o.flexible) {
            k_dot_m<R><<<nb, kWG, 0, st>>>(N, s->r, s->zold, s->partial);
            k_finalize_m<R><<<1, kWG, 0, st>>>(nb, s->partial, s->sc, 5, 0);
        }
        k_dot_m<R><<<nb, kWG, 0, st>>>(N, s->r, s->z, s->partial);
        k_finalize_m<R><<<1, kWG, 0, st>>>(nb, s->partial, s->sc, 3, o.flexible ? 2 : 1);
        k_update_p_m<R><<<blocks_for(NR), kWG, 0, st>>>(NR, s->sc, s->z, s->pv, 0);
    }
    HIPCHK(hipStreamSynchronize(st));   // the last mask upload has completed
    return DGMG_NOT_CONVERGED;
}

#define DISPATCH_R(rval, ...)                                                          \
    switch (rval) {                                                                    \
        case 8: { constexpr int RV = 8; __VA_ARGS__; } break;                          \
        default: fail(DGMG_EINVAL, "unsupported number of right-hand sides");          \
    }

// ------------------------------------------------------------------ setup
static void build_nbr(const BlockOp& A, std::vector<int32_t>& ptr, std::vector<int32_t>& cell,
                      std::vector<int32_t>& code) {
    ptr.assign(A.n + 1, 0);
    for (int64_t f = 0; f < A.nf; ++f) {
        ptr[A.fc[2 * f] + 1]++;
        ptr[A.fc[2 * f + 1] + 1]++;
    }
    for (int64_t K = 0; K < A.n; ++K) ptr[K + 1] += ptr[K];
    cell.assign(ptr[A.n], 0);
    code.assign(ptr[A.n], 0);
    std::vector<int32_t> pos(ptr.begin(), ptr.end() - 1);
    for (int64_t f = 0; f < A.nf; ++f) {
        const int64_t p = A.fc[2 * f], m = A.fc[2 * f + 1];
        cell[pos[p]] = (int32_t)m;
        code[pos[p]++] = (int32_t)(f << 1);
        cell[pos[m]] = (int32_t)p;
        code[pos[m]++] = (int32_t)((f << 1) | 1);
    }
}

// Tile-ELL layout of a level operator (see kernels.hpp): per tile of
// TC = 256/b cells, slot 0 holds the cell blocks and slot r >= 1 the r-th
// neighbour block of every cell, oriented for the row cell and interleaved
// so that the tile's rows are contiguous for each (slot, column).
struct TileEll {
    std::vector<int32_t> slot_ptr, snb;
    std::vector<double> vals;
    std::vector<int32_t> cmap;   // tile position -> cell; empty: identity
};
// Tile-ELL: each tile is padded to its largest neighbour count.  With
// window > 0 the cells of every run of `window` tiles are assigned to tile
// positions by descending neighbour count (stable), so that a tile holds
// cells of similar count while staying among nearby cells; kept only when
// it saves at least 3% of the slots.
static TileEll build_tile_ell(const BlockOp& A, int window = 0) {
    const int b = A.b, TC = kWG / b, TR = TC * b;
    const int64_t n = A.n, ntiles = (n + TC - 1) / TC;
    std::vector<int32_t> ptr, cell, code;
    build_nbr(A, ptr, cell, code);
    auto deg = [&](int64_t c) { return ptr[c + 1] - ptr[c]; };
    std::vector<int32_t> order(n);
    for (int64_t c = 0; c < n; ++c) order[c] = (int32_t)c;
    auto count_slots = [&]() {
        int64_t tot = 0;
        for (int64_t t = 0; t < ntiles; ++t) {
            int mx = 0;
            for (int lc = 0; lc < TC && t * TC + lc < n; ++lc) mx = std::max(mx, deg(order[t * TC + lc]));
            tot += 1 + mx;
        }
        return tot;
    };
    TileEll E;
    if (window > 0) {
        const int64_t plain = count_slots();
        const int64_t w = (int64_t)window * TC;
        for (int64_t w0 = 0; w0 < n; w0 += w)
            std::stable_sort(order.begin() + w0, order.begin() + std::min(n, w0 + w),
                             [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
        if (count_slots() * 100 <= plain * 97)
            E.cmap = order;
        else
            for (int64_t c = 0; c < n; ++c) order[c] = (int32_t)c;
    }
    E.slot_ptr.assign(ntiles + 1, 0);
    for (int64_t t = 0; t < ntiles; ++t) {
        int mx = 0;
        for (int lc = 0; lc < TC; ++lc) {
            const int64_t pos = t * TC + lc;
            if (pos < n) mx = std::max(mx, deg(order[pos]));
        }
        E.slot_ptr[t + 1] = E.slot_ptr[t] + 1 + mx;
    }
    const int64_t nslots = E.slot_ptr[ntiles];
    E.vals.assign((size_t)nslots * b * TR, 0.0);
    E.snb.assign((size_t)nslots * TC, 0);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t s0 = E.slot_ptr[t], ns = E.slot_ptr[t + 1] - s0;
        for (int lc = 0; lc < TC; ++lc) {
            if (t * TC + lc >= n) continue;
            const int64_t c = order[t * TC + lc];
            for (int64_t sl = 0; sl < ns; ++sl) E.snb[(size_t)(s0 + sl) * TC + lc] = (int32_t)c;
            auto put = [&](int64_t gs, const double* blk, bool transpose) {
                for (int i = 0; i < b; ++i)
                    for (int j = 0; j < b; ++j)
                        E.vals[((size_t)gs * b + j) * TR + (size_t)lc * b + i] =
                            transpose ? blk[j * b + i] : blk[i * b + j];
            };
            put(s0, &A.diag[(size_t)c * b * b], false);
            for (int32_t e = ptr[c]; e < ptr[c + 1]; ++e) {
                const int64_t gs = s0 + 1 + (e - ptr[c]);
                E.snb[(size_t)gs * TC + lc] = cell[e];
                put(gs, &A.fblk[(size_t)(code[e] >> 1) * b * b], (code[e] & 1) != 0);
            }
        }
    }
    return E;
}

// Axis-ELL layout of the fine operator (see kernels.hpp): per tile of TC
// cells, the symmetric cell blocks in b/2 + 1 cyclic planes, then b planes
// per axis a of the block A[c, up_a(c)] of the face on the upper a-side of
// each cell; up/lo map every cell to its upper /
// lower neighbour along each axis.  Faces are (plus = lower cell, minus =
// upper cell, axis) as found on the conforming mesh.
struct AxisEll {
    std::vector<int32_t> up, lo;
    std::vector<double> vals;
    bool sparse = false;   // face blocks in the sparse-face form (kernels.hpp)
};
// Whether every face block vanishes outside the rows of the lower cell's
// upper face and the columns of the upper cell's lower face (exact zeros).
static bool faces_are_nodal(const BlockOp& A, const std::vector<int64_t>& upface, int d) {
    const int b = A.b, q = ax_nodes_1d(b, d);
    if (q < 2 || std::pow(q, d) != b) return false;
    const int64_t n = A.n;
    bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int64_t c = 0; c < n; ++c)
        for (int a = 0; a < d; ++a) {
            const int64_t f = upface[(size_t)a * n + c];
            if (f < 0) continue;
            const double* F = &A.fblk[(size_t)f * b * b];
            for (int i = 0; i < b; ++i)
                for (int j = 0; j < b; ++j)
                    if (node_coord(i, a, q) != q - 1 && node_coord(j, a, q) != 0 && F[(size_t)i * b + j] != 0.0)
                        ok = false;
        }
    return ok;
}
// sparse: store the face blocks in the sparse-face form when they are nodal
static AxisEll build_axis_ell(const BlockOp& A, const std::vector<int>& axis, int d, bool with_vals,
                              bool sparse = false) {
    const int b = A.b, TC = kWG / b, TR = TC * b, P0 = ax_cell_planes(b), TP = ax_tile_planes(b, d);
    const int64_t n = A.n, ntiles = (n + TC - 1) / TC;
    if ((int64_t)axis.size() != A.nf) fail(DGMG_EINVAL, "face axis list does not match the operator");
    AxisEll E;
    E.up.resize((size_t)d * n);
    E.lo.assign((size_t)d * n, -1);
    std::vector<int64_t> upface((size_t)d * n, -1);   // face on the upper a-side of each cell
    for (int a = 0; a < d; ++a)
        for (int64_t c = 0; c < n; ++c) E.up[(size_t)a * n + c] = (int32_t)c;
    for (int64_t f = 0; f < A.nf; ++f) {
        const int64_t p = A.fc[2 * f], m = A.fc[2 * f + 1];
        const int a = axis[f];
        if (a < 0 || a >= d) fail(DGMG_EINVAL, "bad face axis");
        if (E.up[(size_t)a * n + p] != p || E.lo[(size_t)a * n + m] != -1)
            fail(DGMG_EUNSUPPORTED, "two faces on one side of a cell");
        E.up[(size_t)a * n + p] = (int32_t)m;
        E.lo[(size_t)a * n + m] = (int32_t)p;
        upface[(size_t)a * n + p] = f;
    }
    if (!with_vals) return E;
    E.sparse = sparse && faces_are_nodal(A, upface, d);
    // per tile: the cell blocks' symmetric planes (plane k, row (cell, i):
    // entry [i][(i + k) mod b]), then per upper face either b planes
    // (plane j, row (cell, i): entry [i][j]) or the sparse-face form
    const int q = ax_nodes_1d(b, d), nF = b / q;
    const int64_t TS = E.sparse ? ax_sparse_tile_values(b, d, TC) : (int64_t)TP * TR;
    const int64_t AXS = ax_sparse_axis_values(b, d, TC);
    E.vals.assign((size_t)(ntiles * TS), 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        const int64_t t = c / TC, lc = c - t * TC;
        const size_t row0 = (size_t)lc * b;
        const double* D = &A.diag[(size_t)c * b * b];
        for (int k = 0; k < P0; ++k)
            for (int i = 0; i < b; ++i)
                E.vals[(size_t)(t * TS) + (size_t)k * TR + row0 + i] = D[(size_t)i * b + (i + k) % b];
        for (int a = 0; a < d; ++a) {
            const int64_t f = upface[(size_t)a * n + c];
            if (f < 0) continue;
            const double* F = &A.fblk[(size_t)f * b * b];
            if (E.sparse) {
                const size_t ab = (size_t)(t * TS) + (size_t)P0 * TR + (size_t)(a * AXS);
                for (int j = 0; j < b; ++j) {
                    const int cj = node_coord(j, a, q), tj = node_tan(j, a, q);
                    if (cj == 0) {
                        for (int i = 0; i < b; ++i) E.vals[ab + (size_t)tj * TR + row0 + i] = F[(size_t)i * b + j];
                    } else {
                        const size_t sp = ab + (size_t)nF * TR + (size_t)(tj * (q - 1) + cj - 1) * TC * nF;
                        for (int i = 0; i < b; ++i)
                            if (node_coord(i, a, q) == q - 1)
                                E.vals[sp + (size_t)lc * nF + node_tan(i, a, q)] = F[(size_t)i * b + j];
                    }
                }
            } else {
                for (int j = 0; j < b; ++j)
                    for (int i = 0; i < b; ++i)
                        E.vals[(size_t)(t * TS) + (size_t)(P0 + a * b + j) * TR + row0 + i] = F[(size_t)i * b + j];
            }
        }
    }
    return E;
}

// Faces of an agglomerated level whose boxes form a conforming grid: every
// face separates its two boxes along one axis (centroid offset above half the
// mean extent along it, below a quarter along the others).  Gives the axis
// and whether the stored plus cell is the upper one; leaves `axis` empty when
// some face does not qualify.
static void coarse_face_axes(const BlockOp& A, const std::vector<double>& lo, const std::vector<double>& hi,
                             int d, std::vector<int>& axis, std::vector<char>& flip) {
    axis.assign(A.nf, -1);
    flip.assign(A.nf, 0);
    for (int64_t f = 0; f < A.nf; ++f) {
        const int64_t p = A.fc[2 * f], m = A.fc[2 * f + 1];
        int best = -1;
        double rbest = 0.0;
        bool aligned = true;
        for (int a = 0; a < d; ++a) {
            const double dc = 0.5 * (lo[m * d + a] + hi[m * d + a]) - 0.5 * (lo[p * d + a] + hi[p * d + a]);
            const double ext = 0.5 * (hi[p * d + a] - lo[p * d + a] + hi[m * d + a] - lo[m * d + a]);
            if (!(ext > 0)) {
                aligned = false;
                break;
            }
            const double r = std::fabs(dc) / ext;
            if (r > rbest) {
                if (best >= 0 && rbest >= 0.25) aligned = false;
                rbest = r;
                best = a;
            } else if (r >= 0.25) {
                aligned = false;
            }
        }
        if (!aligned || best < 0 || rbest <= 0.5) {
            axis.clear();
            flip.clear();
            return;
        }
        const double dcb = 0.5 * (lo[m * d + best] + hi[m * d + best]) - 0.5 * (lo[p * d + best] + hi[p * d + best]);
        axis[f] = best;
        flip[f] = dcb < 0 ? 1 : 0;
    }
}

// prolongation blocks (row-major per fine entity) in tile-interleaved layout
template <typename T>
static std::vector<T> interleave_P(const std::vector<double>& P, int b, int64_t n) {
    const int TC = kWG / b, TR = TC * b;
    const int64_t ntiles = (n + TC - 1) / TC;
    std::vector<T> out((size_t)ntiles * b * TR, (T)0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        const int64_t t = e / TC;
        const int lc = (int)(e - t * TC);
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j)
                out[((size_t)t * b + j) * TR + (size_t)lc * b + i] = (T)P[((size_t)e * b + i) * b + j];
    }
    return out;
}

// Distinct b x b blocks of P (bitwise equal): true, with a type per entity and
// the row-major table of distinct blocks, when there are at most `maxt`.
constexpr int kMaxPTypes = 64;
static bool distinct_blocks(const std::vector<double>& P, int b, int64_t n, int maxt, std::vector<int32_t>& type,
                            std::vector<double>& table) {
    const size_t bb = (size_t)b * b;
    std::vector<uint64_t> h(n);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        uint64_t x = 1469598103934665603ull;   // FNV-1a over the block's bytes
        const unsigned char* c = reinterpret_cast<const unsigned char*>(&P[(size_t)e * bb]);
        for (size_t k = 0; k < bb * sizeof(double); ++k) x = (x ^ c[k]) * 1099511628211ull;
        h[e] = x;
    }
    std::vector<uint64_t> th;
    std::vector<int64_t> rep;
    type.assign(n, -1);
    for (int64_t e = 0; e < n; ++e) {
        int t = -1;
        for (size_t k = 0; k < th.size(); ++k)
            if (th[k] == h[e] &&
                std::memcmp(&P[(size_t)e * bb], &P[(size_t)rep[k] * bb], bb * sizeof(double)) == 0) {
                t = (int)k;
                break;
            }
        if (t < 0) {
            if ((int)th.size() == maxt) return false;
            t = (int)th.size();
            th.push_back(h[e]);
            rep.push_back(e);
        }
        type[e] = t;
    }
    table.resize(rep.size() * bb);
    for (size_t k = 0; k < rep.size(); ++k)
        std::copy(&P[(size_t)rep[k] * bb], &P[(size_t)rep[k] * bb] + bb, &table[k * bb]);
    return true;
}

template <typename T>
static std::vector<T> convert(const std::vector<double>& a) {
    std::vector<T> out(a.size());
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < a.size(); ++k) out[k] = (T)a[k];
    return out;
}

// Fills the strict upper triangle (column-major view) of an n x n matrix
// from its lower triangle.
__global__ void k_symmetrize(int32_t n, double* __restrict__ a) {
    const int i = blockIdx.x * kWG + threadIdx.x;   // row
    const int j = blockIdx.y;                       // column
    if (i < j && j < n) a[(size_t)j * n + i] = a[(size_t)i * n + j];
}

// Dense SPD inverse on the device (set-up only): Cholesky factorisation and
// inverse from the factor with rocSOLVER, then symmetrisation.  A is
// symmetric, so row- and column-major storage coincide.
static double* device_spd_inverse(dgmg_solver* s, const std::vector<double>& a, int64_t n) {
    double* d = s->upload(a);
    int* info = s->dalloc<int>(1);
    rocblas_handle hnd;
    if (rocblas_create_handle(&hnd) != rocblas_status_success) fail(DGMG_EHIP, "rocblas_create_handle failed");
    rocblas_status st1 = rocsolver_dpotrf(hnd, rocblas_fill_lower, (rocblas_int)n, d, (rocblas_int)n, info);
    int h_info = 0;
    HIPCHK(hipMemcpy(&h_info, info, sizeof(int), hipMemcpyDeviceToHost));
    if (st1 != rocblas_status_success) {
        rocblas_destroy_handle(hnd);
        fail(DGMG_EHIP, "rocsolver_dpotrf failed");
    }
    if (h_info != 0) {
        rocblas_destroy_handle(hnd);
        fail(DGMG_ENOTSPD, "coarse operator is not positive definite");
    }
    rocblas_status st2 = rocsolver_dpotri(hnd, rocblas_fill_lower, (rocblas_int)n, d, (rocblas_int)n, info);
    HIPCHK(hipMemcpy(&h_info, info, sizeof(int), hipMemcpyDeviceToHost));
    rocblas_destroy_handle(hnd);
    if (st2 != rocblas_status_success || h_info != 0) fail(DGMG_EHIP, "rocsolver_dpotri failed");
    dim3 g((unsigned)((n + kWG - 1) / kWG), (unsigned)n);
    k_symmetrize<<<g, kWG>>>((int32_t)n, d);
    HIPCHK(hipDeviceSynchronize());
    return d;
}

// Identical axis-aligned boxes: every cell's corners are X_0 + sum_k bit_k h_k e_k
// with the same h (relative tolerance 1e-12).  Returns false otherwise.
static bool uniform_boxes(const Hierarchy& h, double* ext) {
    const int d = h.dim, nc = 1 << d;
    double scale = 0.0;
    for (double v : h.xyz) scale = std::max(scale, std::fabs(v));
    const double tol = 1e-12 * std::max(1.0, scale);
    for (int k = 0; k < d; ++k) {
        const int64_t v0 = h.cells[0], v1 = h.cells[(size_t)1 << k];
        ext[k] = h.xyz[(size_t)v1 * d + k] - h.xyz[(size_t)v0 * d + k];
        if (!(ext[k] > 0)) return false;
    }
    for (int64_t c = 0; c < h.n_cells; ++c) {
        const int64_t* cv = &h.cells[(size_t)c * nc];
        const double* x0 = &h.xyz[(size_t)cv[0] * d];
        for (int corner = 1; corner < nc; ++corner) {
            const double* xc = &h.xyz[(size_t)cv[corner] * d];
            for (int k = 0; k < d; ++k) {
                const double want = x0[k] + (((corner >> k) & 1) ? ext[k] : 0.0);
                if (std::fabs(xc[k] - want) > tol) return false;
            }
        }
    }
    return true;
}

// 1D tables and geometry constants of the matrix-free fine level.
template <typename T>
static MfConst<T> mf_constants(const dgmg_solver* s, const RefElement& re, const T* dev_D) {
    MfConst<T> C{};
    const int Q = re.q;
    std::vector<double> v(Q), dv(Q);
    for (int g = 0; g < Q; ++g) {
        lagrange1d(re.nodes, re.gx[g], v.data(), dv.data());
        for (int j = 0; j < Q; ++j) {
            C.Ig[g * Q + j] = (T)v[j];
            C.Dg[g * Q + j] = (T)dv[j];
        }
        C.gw[g] = (T)re.gw[g];
    }
    for (int e = 0; e < 2; ++e) {
        lagrange1d(re.nodes, (double)e, v.data(), dv.data());
        for (int j = 0; j < Q; ++j) C.Ed[e * Q + j] = (T)dv[j];
    }
    double vol = 1.0;
    for (int k = 0; k < s->dim; ++k) vol *= s->mf_h[k];
    C.vol = (T)vol;
    for (int k = 0; k < s->dim; ++k) {
        C.hinv[k] = (T)(1.0 / s->mf_h[k]);
        C.area[k] = (T)(vol / s->mf_h[k]);
        C.eta[k] = (T)s->mf_eta[k];
    }
    C.cM = (T)s->mf_cM;
    C.D = dev_D;
    return C;
}

static void upload_level(dgmg_solver* s, int l) {
    const BlockOp& A = s->ops[l];
    DevLevel& L = s->lv[l];
    const int b = s->b;
    L.n = (int32_t)A.n;
    L.nf = (int32_t)A.nf;
    L.N = A.n * b;
    std::vector<double> dinv(L.N);
    for (int64_t K = 0; K < A.n; ++K)
        for (int i = 0; i < b; ++i) dinv[K * b + i] = 1.0 / A.diag[((size_t)K * b + i) * b + i];
    const bool last = (l == s->L - 1);
    // the fine level of a conforming mesh is stored once per face (axis-ELL)
    // unless the caller asks for the tile-ELL layout everywhere
    const bool mf = l == 0 && s->fine_layout == DGMG_LAYOUT_MATRIX_FREE;
    const bool ax = l == 0 && !mf && s->fine_layout != DGMG_LAYOUT_TILE_ELL && !s->axis0.empty();
    // agglomerated levels that form a conforming grid of boxes also store each
    // face block once (faces reoriented from the lower to the upper box)
    bool axc = false;
    AxisEll Ec;
    if (l > 0 && !last && s->fine_layout != DGMG_LAYOUT_TILE_ELL && (size_t)l < s->axisl.size() &&
        !s->axisl[l].empty()) {
        BlockOp Ao;
        Ao.n = A.n;
        Ao.b = A.b;
        Ao.nf = A.nf;
        Ao.diag = A.diag;
        Ao.fc = A.fc;
        Ao.fblk = A.fblk;
        const std::vector<char>& fl = s->flipl[l];
        for (int64_t f = 0; f < A.nf; ++f)
            if (fl[f]) {
                std::swap(Ao.fc[2 * f], Ao.fc[2 * f + 1]);
                double* blk = &Ao.fblk[(size_t)f * b * b];
                for (int i = 0; i < b; ++i)
                    for (int j = i + 1; j < b; ++j) std::swap(blk[i * b + j], blk[j * b + i]);
            }
        try {
            Ec = build_axis_ell(Ao, s->axisl[l], s->dim, true);
            axc = true;
        } catch (const Error& e) {
            if (e.code != DGMG_EUNSUPPORTED) throw;   // two faces on one side: keep tile-ELL
        }
    }
    if (mf) {
        // neighbours as in the axis-ELL layout; no operator values are stored
        AxisEll E = build_axis_ell(A, s->axis0, s->dim, false);
        L.mf = true;
        L.up = s->upload(E.up);
        L.lo = s->upload(E.lo);
        L.dinv64 = s->upload(dinv);
        RefElement re;
        re.init(s->dim, s->p);
        L.mf64 = mf_constants<double>(s, re, s->upload(s->mf_D));
        if (s->prec == DGMG_PREC_MIXED) {
            L.dinv32 = s->upload(convert<float>(dinv));
            L.mf32 = mf_constants<float>(s, re, s->upload(convert<float>(s->mf_D)));
        }
    } else if (ax || axc) {
        // single-column solvers store nodal fine face blocks in sparse form
        // (the multi-column kernels read whole blocks)
        const bool sparse = !axc && s->max_rhs <= 1 && s->fine_layout != DGMG_LAYOUT_AXIS_ELL_DENSE;
        AxisEll E = axc ? std::move(Ec) : build_axis_ell(A, s->axis0, s->dim, true, sparse);
        L.ax = true;
        L.sf = E.sparse;
        L.up = s->upload(E.up);
        L.lo = s->upload(E.lo);
        L.vals64 = s->upload(E.vals);
        L.dinv64 = s->upload(dinv);
        if (s->prec == DGMG_PREC_MIXED) {
            L.vals32 = s->upload(convert<float>(E.vals));
            L.dinv32 = s->upload(convert<float>(dinv));
        }
    } else if (!last || s->L == 1) {
        // single-column solvers group cells of similar neighbour count
        // into tiles (the multi-column kernels keep the identity mapping)
        TileEll E = build_tile_ell(A, s->max_rhs == 1 ? 16 : 0);
        if (!E.cmap.empty()) L.cmap = s->upload(E.cmap);
        L.slot_ptr = s->upload(E.slot_ptr);
        L.snb = s->upload(E.snb);
        L.vals64 = s->upload(E.vals);
        L.dinv64 = s->upload(dinv);
        if (s->prec == DGMG_PREC_MIXED) {
            L.vals32 = s->upload(convert<float>(E.vals));
            L.dinv32 = s->upload(convert<float>(dinv));
        }
    }
    if (!last && s->jacobi == DGMG_JACOBI_CELL_BLOCK) {
        L.bj64 = s->upload(s->bjinv[l]);
        if (s->prec == DGMG_PREC_MIXED) L.bj32 = s->upload(convert<float>(s->bjinv[l]));
        std::vector<double>().swap(s->bjinv[l]);
    }
    if (!last) {
        std::vector<int32_t> par(s->parents[l].begin(), s->parents[l].end());
        L.parent = s->upload(par);
        std::vector<int32_t> ptype;
        std::vector<double> ptab;
        if (distinct_blocks(s->Ph[l], b, A.n, kMaxPTypes, ptype, ptab)) {
            // few distinct prolongation blocks (boxes nested in boxes): a table
            // of them and a type per entity instead of one block each.  The
            // table holds every block row-major (read by the restriction,
            // lanes along a column), then every block transposed (read by
            // the prolongation, lanes along a row).
            L.ptype = s->upload(ptype);
            const size_t bb = (size_t)b * b;
            L.ntypes = (int32_t)(ptab.size() / bb);
            ptab.resize(2 * L.ntypes * bb);
            for (int32_t q = 0; q < L.ntypes; ++q)
                for (int i = 0; i < b; ++i)
                    for (int j = 0; j < b; ++j) ptab[(L.ntypes + q) * bb + (size_t)j * b + i] = ptab[q * bb + (size_t)i * b + j];
            L.P64 = s->upload(ptab);
            if (s->prec == DGMG_PREC_MIXED) L.P32 = s->upload(convert<float>(ptab));
        } else {
            L.P64 = s->upload(interleave_P<double>(s->Ph[l], b, A.n));
            if (s->prec == DGMG_PREC_MIXED) L.P32 = s->upload(interleave_P<float>(s->Ph[l], b, A.n));
        }
    }
    if (l > 0) {
        const auto& par = s->parents[l - 1];
        std::vector<int32_t> cp(A.n + 1, 0), cl(par.size());
        for (auto K : par) cp[K + 1]++;
        for (int64_t K = 0; K < A.n; ++K) cp[K + 1] += cp[K];
        std::vector<int32_t> pos(cp.begin(), cp.end() - 1);
        for (size_t e = 0; e < par.size(); ++e) cl[pos[par[e]]++] = (int32_t)e;
        L.child_ptr = s->upload(cp);
        L.child_list = s->upload(cl);
    }
    const size_t es = s->prec == DGMG_PREC_MIXED ? sizeof(float) : sizeof(double);
    auto vec = [&]() -> void* { return (void*)s->dalloc<char>(L.N * s->max_rhs * es); };
    L.vb = vec(); L.vx = vec(); L.vx2 = vec(); L.vr = vec(); L.vd = vec(); L.vd2 = vec();
}

}  // namespace dgmg

// ====================================================================== C ABI
// Number of block partials the single-column PCG reduces (the larger of the
// vector kernels' and the level-0 block kernels' workgroup counts, plus slack).
static int64_t pcg_partials(const dgmg_solver* s) {
    return (int64_t)std::max(blocks_for(s->N), level_tiles<double>(s, s->lv[0])) + 16;
}

// ------------------------------------------------- static PCG scratch
// Reduction scratch of dgmg_pcg_solve_noalloc: the 8 scalar slots of pcg()
// at offset 0 and its block partials from kScratchPartial on.  A file-scope
// device array: every GPU the library runs on holds its own copy, at its own
// address, until the process ends.  Host code never passes `scratch` itself
// (in host code the name is a stand-in, not a device address); it uses the
// address hipGetSymbolAddress returns for the device, resolved once per
// device at set-up.
constexpr int64_t kScratchDoubles = 131072;   // 1 MiB per GPU
constexpr int64_t kScratchPartial = 32;       // partials start 256 bytes in
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxScratchDevices] = {};

// Address of `scratch` on the current device (resolved on the first call
// for that device, with it current).
static double* scratch_address() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) fail(DGMG_EUNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(DGMG_EHIP, "hipGetSymbolAddress returned a null address for the PCG scratch");
        g_scratch_dev[dev] = (double*)p;
    }
    return g_scratch_dev[dev];
}

#define API_BEGIN try {
#define API_END                                                          \
    }                                                                    \
    catch (const Error& e) {                                             \
        set_last_error(e.msg);                                           \
        return e.code;                                                   \
    }                                                                    \
    catch (const std::bad_alloc&) {                                      \
        set_last_error("out of host memory");                            \
        return DGMG_ENOMEM;                                              \
    }                                                                    \
    catch (const std::exception& e) {                                    \
        set_last_error(e.what());                                        \
        return DGMG_EINVAL;                                              \
    }

// Sort-tile-recursive packing of items with boxes (lo, hi) into groups of at
// most M: with P = ceil(N/M) and S the smallest integer with S^d >= P, sort
// by centre x into slabs of S^(d-1) M items, each slab by y into strips of
// S M items (3D), each strip by z, then cut consecutive runs of M.  Ties are
// broken by item id.  Returns the number of groups; par receives each
// item's group (numbered in packing order).
static int64_t str_pack(const std::vector<double>& lo, const std::vector<double>& hi, int d, int M,
                        std::vector<int64_t>& par) {
    const int64_t N = (int64_t)(lo.size() / d);
    const int64_t P = (N + M - 1) / M;
    int64_t S = 1;
    auto pw = [&](int64_t v) { int64_t r = 1; for (int k = 0; k < d; ++k) r *= v; return r; };
    while (pw(S) < P) ++S;
    auto cen = [&](int64_t i, int a) { return 0.5 * (lo[(size_t)i * d + a] + hi[(size_t)i * d + a]); };
    auto by = [&](int a) {
        return [&, a](int64_t x, int64_t y) {
            const double cx = cen(x, a), cy = cen(y, a);
            return cx < cy || (cx == cy && x < y);
        };
    };
    std::vector<int64_t> order(N);
    for (int64_t i = 0; i < N; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), by(0));
    par.assign(N, -1);
    int64_t g = 0;
    const int64_t slab = pw(S) / S * M;
    for (int64_t a0 = 0; a0 < N; a0 += slab) {
        const int64_t a1 = std::min(N, a0 + slab);
        std::sort(order.begin() + a0, order.begin() + a1, by(1));
        auto cut = [&](int64_t r0, int64_t r1) {
            for (int64_t c = r0; c < r1; c += M) {
                for (int64_t k = c; k < std::min(r1, c + M); ++k) par[order[k]] = g;
                ++g;
            }
        };
        if (d == 3) {
            const int64_t strip = S * M;
            for (int64_t b0 = a0; b0 < a1; b0 += strip) {
                const int64_t b1 = std::min(a1, b0 + strip);
                std::sort(order.begin() + b0, order.begin() + b1, by(2));
                cut(b0, b1);
            }
        } else {
            cut(a0, a1);
        }
    }
    return g;
}

extern "C" {

const char* dgmg_last_error(void) { return g_last_error.c_str(); }

int dgmg_build_hierarchy(const dgmg_mesh* m, const dgmg_agglo_opts* o, dgmg_hierarchy** out) {
    API_BEGIN
    if (!m || !o || !out || !m->xyz || !m->cell_vtx) fail(DGMG_EINVAL, "null argument");
    if (m->dim != 2 && m->dim != 3) fail(DGMG_EUNSUPPORTED, "dimension must be 2 or 3");
    if (m->n_cells <= 0 || m->n_vert <= 0) fail(DGMG_EINVAL, "empty mesh");
    if (o->n_levels < 1 || o->n_levels > DGMG_MAX_LEVELS) fail(DGMG_EINVAL, "bad number of levels");
    auto* h = new dgmg_hierarchy();
    std::unique_ptr<dgmg_hierarchy> guard(h);
    const int d = m->dim, nc = 1 << d;
    h->dim = d;
    h->n_vert = m->n_vert;
    h->n_cells = m->n_cells;
    h->xyz.assign(m->xyz, m->xyz + (size_t)m->n_vert * d);
    h->cells.assign(m->cell_vtx, m->cell_vtx + (size_t)m->n_cells * nc);
    for (auto v : h->cells)
        if (v < 0 || v >= m->n_vert) fail(DGMG_EINVAL, "vertex id out of range");
    h->n_levels = o->n_levels;
    h->n_ent.assign(1, m->n_cells);
    if (o->method == DGMG_AGGLO_GRID) {
        double lo[3], hi[3];
        for (int a = 0; a < d; ++a) {
            lo[a] = INFINITY;
            hi[a] = -INFINITY;
        }
        for (int64_t v = 0; v < m->n_vert; ++v)
            for (int a = 0; a < d; ++a) {
                lo[a] = std::min(lo[a], h->xyz[(size_t)v * d + a]);
                hi[a] = std::max(hi[a], h->xyz[(size_t)v * d + a]);
            }
        std::vector<double> cen((size_t)h->n_cells * d, 0.0);
        for (int64_t c = 0; c < h->n_cells; ++c)
            for (int k = 0; k < nc; ++k)
                for (int a = 0; a < d; ++a) cen[(size_t)c * d + a] += h->xyz[(size_t)h->cells[(size_t)c * nc + k] * d + a];
        for (auto& v : cen) v /= nc;
        std::vector<int64_t> prev_id(h->n_cells);  // level-(l-1) id of each fine cell
        for (int64_t c = 0; c < h->n_cells; ++c) prev_id[c] = c;
        for (int l = 1; l < o->n_levels; ++l) {
            int64_t nbins = 1;
            for (int a = 0; a < d; ++a) {
                if (o->grid_bins[l][a] < 1) fail(DGMG_EINVAL, "grid_bins must be >= 1");
                nbins *= o->grid_bins[l][a];
            }
            std::vector<int64_t> id(h->n_cells);
            for (int64_t c = 0; c < h->n_cells; ++c) {
                int64_t lin = 0;
                for (int a = d - 1; a >= 0; --a) {
                    const int nb = o->grid_bins[l][a];
                    int64_t k = (int64_t)std::floor((cen[(size_t)c * d + a] - lo[a]) / (hi[a] - lo[a]) * nb);
                    k = std::min<int64_t>(std::max<int64_t>(k, 0), nb - 1);
                    lin = lin * nb + k;
                }
                id[c] = lin;
            }
            std::vector<int64_t> par(h->n_ent[l - 1], -1);
            std::vector<char> used(nbins, 0);
            for (int64_t c = 0; c < h->n_cells; ++c) {
                int64_t& pp = par[prev_id[c]];
                if (pp >= 0 && pp != id[c]) fail(DGMG_EINVAL, "grid bins do not nest across levels");
                pp = id[c];
                used[id[c]] = 1;
            }
            for (int64_t k = 0; k < nbins; ++k)
                if (!used[k]) fail(DGMG_EINVAL, "empty agglomerate (grid bin without cells)");
            h->parent.push_back(par);
            h->n_ent.push_back(nbins);
            prev_id = id;
        }
    } else if (o->method == DGMG_AGGLO_RTREE_STR) {
        // STR bulk-loaded R-tree: level l+1 packs the bounding boxes of level l
        // (Algorithms 1 and 2 on a sort-tile-recursive tree)
        const int M = o->rtree_fanout;
        if (M < 2) fail(DGMG_EINVAL, "rtree_fanout must be >= 2");
        std::vector<double> lo((size_t)h->n_cells * d), hi((size_t)h->n_cells * d);
        for (int64_t c = 0; c < h->n_cells; ++c)
            for (int a = 0; a < d; ++a) {
                double mn = INFINITY, mx = -INFINITY;
                for (int k = 0; k < nc; ++k) {
                    const double x = h->xyz[(size_t)h->cells[(size_t)c * nc + k] * d + a];
                    mn = std::min(mn, x);
                    mx = std::max(mx, x);
                }
                lo[(size_t)c * d + a] = mn;
                hi[(size_t)c * d + a] = mx;
            }
        for (int l = 1; l < o->n_levels; ++l) {
            std::vector<int64_t> par;
            const int64_t ngrp = str_pack(lo, hi, d, M, par);
            std::vector<double> nlo((size_t)ngrp * d, INFINITY), nhi((size_t)ngrp * d, -INFINITY);
            for (size_t e = 0; e < par.size(); ++e)
                for (int a = 0; a < d; ++a) {
                    nlo[(size_t)par[e] * d + a] = std::min(nlo[(size_t)par[e] * d + a], lo[e * d + a]);
                    nhi[(size_t)par[e] * d + a] = std::max(nhi[(size_t)par[e] * d + a], hi[e * d + a]);
                }
            h->parent.push_back(par);
            h->n_ent.push_back(ngrp);
            lo.swap(nlo);
            hi.swap(nhi);
        }
    } else if (o->method == DGMG_AGGLO_USER) {
        if (!o->user_parents) fail(DGMG_EINVAL, "user_parents is null");
        for (int l = 1; l < o->n_levels; ++l) {
            const int64_t* up = o->user_parents[l - 1];
            std::vector<int64_t> par(up, up + h->n_ent[l - 1]);
            int64_t mx = -1;
            for (auto v : par) {
                if (v < 0) fail(DGMG_EINVAL, "negative parent id");
                mx = std::max(mx, v);
            }
            std::vector<char> used(mx + 1, 0);
            for (auto v : par) used[v] = 1;
            for (auto u : used)
                if (!u) fail(DGMG_EINVAL, "parent ids are not contiguous");
            h->parent.push_back(par);
            h->n_ent.push_back(mx + 1);
        }
    } else {
        fail(DGMG_EUNSUPPORTED, "agglomeration method not available");
    }
    *out = guard.release();
    return DGMG_OK;
    API_END
}

int dgmg_hierarchy_info(const dgmg_hierarchy* h, int32_t level, int32_t* n_levels, int64_t* n_ent) {
    API_BEGIN
    if (!h) fail(DGMG_EINVAL, "null hierarchy");
    if (n_levels) *n_levels = h->n_levels;
    if (n_ent) {
        if (level < 0 || level >= h->n_levels) fail(DGMG_EINVAL, "level out of range");
        *n_ent = h->n_ent[level];
    }
    return DGMG_OK;
    API_END
}

int dgmg_hierarchy_parents(const dgmg_hierarchy* h, int32_t level, int64_t* out) {
    API_BEGIN
    if (!h || !out) fail(DGMG_EINVAL, "null argument");
    if (level < 0 || level >= h->n_levels - 1) fail(DGMG_EINVAL, "level out of range");
    std::copy(h->parent[level].begin(), h->parent[level].end(), out);
    return DGMG_OK;
    API_END
}

int dgmg_hierarchy_boxes(const dgmg_hierarchy* h, int32_t level, double* lo, double* hi) {
    API_BEGIN
    if (!h || !lo || !hi) fail(DGMG_EINVAL, "null argument");
    if (level < 0 || level >= h->n_levels) fail(DGMG_EINVAL, "level out of range");
    std::vector<double> l, u;
    level_boxes(*h, level, l, u);
    std::copy(l.begin(), l.end(), lo);
    std::copy(u.begin(), u.end(), hi);
    return DGMG_OK;
    API_END
}

void dgmg_destroy_hierarchy(dgmg_hierarchy* h) { delete h; }

int dgmg_setup_levels(const dgmg_hierarchy* h, const dgmg_disc* disc, const dgmg_physics* ph,
                      const dgmg_mg_opts* mg, dgmg_solver** out) {
    API_BEGIN
    if (!h || !disc || !ph || !mg || !out) fail(DGMG_EINVAL, "null argument");
    if (!ph->D_cell) fail(DGMG_EINVAL, "D_cell is null");
    if (!(ph->dt > 0) || !(ph->chi > 0) || !(ph->Cm > 0)) fail(DGMG_EINVAL, "dt, chi, Cm must be > 0");
    if (ph->bdf != 1 && ph->bdf != 2) fail(DGMG_EINVAL, "bdf must be 1 or 2");
    if (mg->cheb_degree < 1 || mg->cheb_sweeps < 0) fail(DGMG_EINVAL, "bad Chebyshev options");
    if (ph->model < 0 || ph->model > 2) fail(DGMG_EINVAL, "unknown ionic model");
    const int need[3] = {4, 3, 28};
    if (ph->n_params != need[ph->model] || !ph->params) fail(DGMG_EINVAL, "wrong number of ionic parameters");
    auto* s = new dgmg_solver();
    std::unique_ptr<dgmg_solver> guard(s);
    RefElement re;
    re.init(h->dim, disc->p);
    s->dim = h->dim;
    s->p = disc->p;
    s->b = re.b;
    s->L = h->n_levels;
    s->prec = mg->precision;
    s->bdf = ph->bdf;
    {
        const char* rx = std::getenv("DGMG_ROCTX");
        s->roctx = rx && rx[0] == '1';
    }
    s->cheb_k = mg->cheb_degree;
    s->cheb_s = mg->cheb_sweeps;
    if (mg->max_rhs != 0 && mg->max_rhs != 1 && mg->max_rhs != DGMG_MULTI_RHS)
        fail(DGMG_EINVAL, "max_rhs must be 0, 1 or DGMG_MULTI_RHS");
    s->max_rhs = mg->max_rhs > 1 ? mg->max_rhs : 1;
    s->mfma = mg->mfma ? 1 : 0;
    if (mg->fine_layout < DGMG_LAYOUT_AUTO || mg->fine_layout > DGMG_LAYOUT_AXIS_ELL_DENSE)
        fail(DGMG_EINVAL, "unknown fine_layout");
    if (mg->fine_layout == DGMG_LAYOUT_MATRIX_FREE && mg->max_rhs > 1)
        fail(DGMG_EUNSUPPORTED, "the matrix-free fine level has no multi-column kernels");
    s->fine_layout = mg->fine_layout;
    if (mg->jacobi != DGMG_JACOBI_POINT && mg->jacobi != DGMG_JACOBI_CELL_BLOCK) fail(DGMG_EINVAL, "unknown jacobi");
    if (mg->jacobi == DGMG_JACOBI_CELL_BLOCK && s->max_rhs > 1)
        fail(DGMG_EUNSUPPORTED, "cell-block Jacobi is implemented for single-column solvers");
    s->jacobi = mg->jacobi;
    s->N = h->n_cells * re.b;
    s->S = ph->model == DGMG_MODEL_BO ? 3 : 1;
    s->parents = h->parent;
    const double cM = (ph->bdf == 2 ? 1.5 : 1.0) * ph->chi * ph->Cm / ph->dt;
    s->cU = ph->bdf == 2 ? ph->chi * ph->Cm / (2.0 * ph->dt) : ph->chi * ph->Cm / ph->dt;
    s->ip.model = ph->model;
    s->ip.S = s->S;
    s->ip.bdf = ph->bdf;
    s->ip.dt = ph->dt;
    s->ip.chi = ph->chi;
    s->ip.Cm = ph->Cm;
    for (int k = 0; k < ph->n_params; ++k) s->ip.p[k] = ph->params[k];

    double t0 = now_s();
    // assembly, prolongation blocks, Galerkin products and Lanczos estimates
    // on the GPU (the adjoint's conductivity derivatives come from the host
    // assembly)
    if (mg->allocator) {
        if (!mg->allocator->alloc || !mg->allocator->free) fail(DGMG_EINVAL, "allocator without alloc or free");
        s->mem.user = *mg->allocator;
        s->mem.has_user = true;
    }
    std::unique_ptr<DeviceSetup> ds;
    if (mg->setup_on_device) {
        if (!mg->device_setup) fail(DGMG_EINVAL, "setup_on_device needs device_setup");
        ds.reset(new DeviceSetup(*h, re, s->mem));
    }
    Faces F = find_faces(*h);
    s->axis0 = F.axis;
    s->ops.resize(s->L);
    AdjointBlocks adj;
    const bool want_adj = mg->adjoint != 0;
    if (want_adj && ph->model == DGMG_MODEL_BO)
        fail(DGMG_EUNSUPPORTED, "the adjoint is implemented for the FHN and Aliev-Panfilov models");
    if (ds && !want_adj)
        ds->assemble_fine(F, re, *disc, *ph, cM, s->ops[0], s->mass_h);
    else
        assemble_fine(*h, F, re, *disc, *ph, cM, s->ops[0], s->mass_h, want_adj ? &adj : nullptr);
    // AUTO: matrix-free on meshes of identical boxes for p >= 2 (single-column
    // solvers), the axis-ELL blocks otherwise
    if (s->fine_layout == DGMG_LAYOUT_AUTO && s->p >= 2 && s->max_rhs == 1 && uniform_boxes(*h, s->mf_h))
        s->fine_layout = DGMG_LAYOUT_MATRIX_FREE;
    if (s->fine_layout == DGMG_LAYOUT_MATRIX_FREE) {
        if (!uniform_boxes(*h, s->mf_h))
            fail(DGMG_EUNSUPPORTED, "the matrix-free fine level needs identical axis-aligned box cells");
        s->mf_cM = cM;
        for (int k = 0; k < s->dim; ++k)
            s->mf_eta[k] = disc->penalty_mode == DGMG_PENALTY_FIXED
                               ? disc->eta
                               : (disc->eta > 0 ? disc->eta : 1.0) * disc->p * (disc->p + 1) / s->mf_h[k];
        const int np = s->dim * (s->dim + 1) / 2;
        s->mf_D.assign(ph->D_cell, ph->D_cell + (size_t)h->n_cells * np);
        if (ph->cell_scale)
            for (int64_t c = 0; c < h->n_cells; ++c)
                for (int k = 0; k < np; ++k) s->mf_D[(size_t)c * np + k] *= ph->cell_scale[c];
    }
    double t1 = now_s();
    s->info.t_assembly = t1 - t0;
    // boxes and prolongations
    std::vector<std::vector<double>> lo(s->L), hi(s->L);
    for (int l = 1; l < s->L; ++l) level_boxes(*h, l, lo[l], hi[l]);
    double t2 = now_s();
    s->info.t_hierarchy = t2 - t1;
    s->Ph.resize(s->L);
    for (int l = 0; l + 1 < s->L; ++l) {
        if (ds)
            ds->prolongation(l, lo[l], hi[l], lo[l + 1], hi[l + 1], s->Ph[l]);
        else
            prolongation_blocks(*h, re, l, lo[l], hi[l], lo[l + 1], hi[l + 1], s->Ph[l]);
    }
    double t3 = now_s();
    s->info.t_transfer = t3 - t2;
    if (ds && s->L > 1) ds->set_fine(s->ops[0]);
    for (int l = 0; l + 1 < s->L; ++l) {
        if (ds)
            ds->galerkin(l, s->ops[l], s->ops[l + 1]);
        else
            galerkin(s->ops[l], s->Ph[l], h->parent[l], h->n_ent[l + 1], s->ops[l + 1]);
    }
    // face axes of agglomerated levels that form a conforming grid of boxes
    s->axisl.assign(s->L, {});
    s->flipl.assign(s->L, {});
    for (int l = 1; l + 1 < s->L; ++l) coarse_face_axes(s->ops[l], lo[l], hi[l], s->dim, s->axisl[l], s->flipl[l]);
    double t4 = now_s();
    s->info.t_galerkin = t4 - t3;
    s->lv.resize(s->L);
    if (s->jacobi == DGMG_JACOBI_CELL_BLOCK) s->bjinv.assign(s->L, {});
    for (int l = 0; l + 1 < s->L; ++l) {
        std::vector<double> chol;
        if (s->jacobi == DGMG_JACOBI_CELL_BLOCK) cell_block_factors(s->ops[l], chol, s->bjinv[l]);
        if (mg->lam_override) {
            s->lv[l].lam_lo = mg->lam_override[2 * l];
            s->lv[l].lam_hi = mg->lam_override[2 * l + 1];
        } else {
            // the block variant's estimate runs on the host (its scaling is a
            // per-cell triangular solve)
            const double th = s->jacobi == DGMG_JACOBI_CELL_BLOCK
                                  ? lanczos_theta_max(s->ops[l], mg->lanczos_steps, &chol)
                                  : ds ? ds->lanczos_theta_max(l, s->ops[l], mg->lanczos_steps)
                                       : lanczos_theta_max(s->ops[l], mg->lanczos_steps);
            s->lv[l].lam_hi = mg->lam_safety * th;
            s->lv[l].lam_lo = s->lv[l].lam_hi / mg->smooth_range;
        }
        if (!(s->lv[l].lam_hi > s->lv[l].lam_lo) || !(s->lv[l].lam_lo > 0))
            fail(DGMG_EINVAL, "invalid Chebyshev interval");
    }
    ds.reset();
    double t5 = now_s();
    s->info.t_smoother = t5 - t4;
    std::vector<double> Ac;
    dense_from_blocks(s->ops[s->L - 1], Ac);
    s->nc_dofs = s->ops[s->L - 1].n * s->b;
    // large coarse problems are factorised on the device (set-up only)
    const bool coarse_on_device = mg->device_setup && s->nc_dofs > kHostCholeskyMax;
    if (!coarse_on_device) {
        if (s->nc_dofs > kHostCholeskyMax)
            fail(DGMG_EUNSUPPORTED, "coarse problem too large for the host factorisation");
        cholesky_inverse(Ac, s->nc_dofs);
    }
    double t6 = now_s();
    s->info.t_coarse = t6 - t5;

    // info
    s->info.dim = s->dim;
    s->info.p = s->p;
    s->info.b = s->b;
    s->info.n_levels = s->L;
    s->info.precision = s->prec;
    s->info.model = ph->model;
    s->info.n_gates = s->S;
    s->info.n_dofs = s->N;
    double nnz0 = 0, nnz = 0;
    for (int l = 0; l < s->L; ++l) {
        s->info.n_cells[l] = s->ops[l].n;
        s->info.n_faces[l] = s->ops[l].nf;
        s->info.lam_lo[l] = s->lv[l].lam_lo;
        s->info.lam_hi[l] = s->lv[l].lam_hi;
        double z = (double)(s->ops[l].n + 2 * s->ops[l].nf) * s->b * s->b;
        if (l == 0) nnz0 = z;
        nnz += z;
    }
    s->info.op_complexity = nnz / nnz0;

    if (mg->device_setup) {
        for (int l = 0; l < s->L; ++l) upload_level(s, l);
        s->Ainv = coarse_on_device ? device_spd_inverse(s, Ac, s->nc_dofs) : s->upload(Ac);
        if (s->prec == DGMG_PREC_MIXED) {
            // the FP32 V-cycle streams the inverse rounded to FP32 (half the
            // bytes of the GEMV; the sums stay in FP64); the FP64 copy goes
            const int64_t nn = s->nc_dofs * s->nc_dofs;
            s->Ainv32 = s->dalloc<float>((size_t)nn);
            k_cast<double, float><<<blocks_for(nn), kWG>>>(nn, s->Ainv, nullptr, s->Ainv32);
            HIPCHK(hipGetLastError());
            HIPCHK(hipDeviceSynchronize());
            s->dfree(s->Ainv, (size_t)nn * sizeof(double));
            s->Ainv = nullptr;
        }
        const int64_t N = s->N, R = s->max_rhs;
        s->r = s->dalloc<double>(N * R);
        s->z = s->dalloc<double>(N * R);
        s->zold = s->dalloc<double>(N * R);
        s->pv = s->dalloc<double>(N * R);
        s->q = s->dalloc<double>(N * R);
        s->bwork = s->dalloc<double>(N * R);
        s->tmp64a = s->dalloc<double>(N);
        s->tmp64b = s->dalloc<double>(N);
        s->partial = s->dalloc<double>(pcg_partials(s) * R);
        s->scratch = scratch_address();
        s->sc = s->dalloc<double>(8 * R);
        HIPCHK(hipMemset(s->sc, 0, 8 * R * sizeof(double)));
        HIPCHK(hipHostMalloc((void**)&s->sc_host, 8 * R * sizeof(double), hipHostMallocMapped));
        HIPCHK(hipHostGetDevicePointer((void**)&s->sc_host_dev, s->sc_host, 0));
        s->act = s->dalloc<int32_t>(R);
        HIPCHK(hipHostMalloc((void**)&s->act_host, R * sizeof(int32_t), hipHostMallocDefault));
        s->mass = s->upload(to_colmajor<double>(s->mass_h, s->b));
        if (want_adj) {
            const int b = s->b, R = 2 * b;
            const BlockOp& A = s->ops[0];
            std::vector<double> Sc(adj.S.size());
            for (int64_t K = 0; K < A.n; ++K)
                for (int i = 0; i < b; ++i)
                    for (int j = 0; j < b; ++j)
                        Sc[((size_t)K * b + j) * b + i] = adj.S[((size_t)K * b + i) * b + j];
            std::vector<double> Xc(adj.X.size());
            for (size_t blk = 0; blk < adj.X.size() / ((size_t)R * R); ++blk)
                for (int I = 0; I < R; ++I)
                    for (int J = 0; J < R; ++J)
                        Xc[(blk * R + J) * R + I] = adj.X[(blk * R + I) * R + J];
            s->adjS = s->upload(Sc);
            s->adjX = s->upload(Xc);
            s->adj_fc = s->upload(A.fc);
            std::vector<int32_t> ptr, cell, code;
            build_nbr(A, ptr, cell, code);
            s->adj_nptr = s->upload(ptr);
            s->adj_ncode = s->upload(code);
            s->nf0 = A.nf;
            s->adjq = s->dalloc<double>(2 * (size_t)A.nf + 2);
            s->has_adjoint = true;
        }
        HIPCHK(hipDeviceSynchronize());
        s->on_device = true;
    }
    s->info.t_upload = now_s() - t6;
    s->info.device_bytes = s->dev_bytes;
    for (int l = 0; l < s->L; ++l) {
        const DevLevel& Lv = s->lv[l];
        s->info.level_layout[l] = !s->on_device || (l == s->L - 1 && s->L > 1) ? 0
                                  : Lv.mf ? DGMG_LAYOUT_MATRIX_FREE
                                  : Lv.ax ? DGMG_LAYOUT_AXIS_ELL : DGMG_LAYOUT_TILE_ELL;
    }
    s->info.fine_layout = s->info.level_layout[0];
    for (int l = 0; l < s->L; ++l) s->info.prolong_types[l] = s->on_device ? s->lv[l].ntypes : 0;
    for (int l = 0; l < s->L; ++l) s->info.level_grouped[l] = s->on_device && s->lv[l].cmap ? 1 : 0;
    s->info.sparse_faces = s->on_device && s->L > 0 && s->lv[0].sf ? 1 : 0;
    *out = guard.release();
    return DGMG_OK;
    API_END
}

void dgmg_destroy_solver(dgmg_solver* s) { delete s; }

int dgmg_get_info(const dgmg_solver* s, dgmg_solver_info* info) {
    API_BEGIN
    if (!s || !info) fail(DGMG_EINVAL, "null argument");
    *info = s->info;
    return DGMG_OK;
    API_END
}

static void need_device(const dgmg_solver* s) {
    if (!s) fail(DGMG_EINVAL, "null solver");
    if (!s->on_device) fail(DGMG_EINVAL, "solver was set up without device data");
}

int dgmg_pcg_solve(dgmg_solver* s, const double* b, double* x, const dgmg_pcg_opts* o,
                   dgmg_pcg_stats* st, void* stream) {
    API_BEGIN
    need_device(s);
    if (!b || !x || !o || !st) fail(DGMG_EINVAL, "null argument");
    return pcg(s, b, x, *o, st, (hipStream_t)stream, s->partial, s->sc);
    API_END
}

int dgmg_pcg_solve_noalloc(dgmg_solver* s, const double* b, double* x, const dgmg_pcg_opts* o,
                           dgmg_pcg_stats* st, void* stream) {
    API_BEGIN
    need_device(s);
    if (!b || !x || !o || !st) fail(DGMG_EINVAL, "null argument");
    const int64_t need = kScratchPartial + pcg_partials(s);
    if (need > kScratchDoubles)
        fail(DGMG_EINVAL, "dgmg_pcg_solve_noalloc: this solver needs " + std::to_string(need) +
                              " doubles of reduction scratch; the static array holds " +
                              std::to_string(kScratchDoubles) + " (use dgmg_pcg_solve)");
    if (!s->scratch) fail(DGMG_EINVAL, "the static PCG scratch was not resolved at set-up");
    hipStream_t hs = (hipStream_t)stream;
    // the array keeps the previous call's contents: clear the scalar slots
    // with a fill kernel (every partial is written before it is read)
    k_fill<double><<<1, kWG, 0, hs>>>(kScratchPartial, s->scratch, 0.0);
    HIPCHK(hipGetLastError());
    return pcg(s, b, x, *o, st, hs, s->scratch + kScratchPartial, s->scratch);
    API_END
}

int dgmg_ionic_step(dgmg_solver* s, const double* U, const double* Up, const double* W,
                    const double* Wp, double* Wn, double* g, void* stream) {
    API_BEGIN
    need_device(s);
    if (!U || !Up || !W || !Wp || !Wn || !g) fail(DGMG_EINVAL, "null argument");
    k_ionic<<<blocks_for(s->N), 256, 0, (hipStream_t)stream>>>(s->N, s->ip, U, Up, W, Wp, Wn, g);
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_time_step(dgmg_solver* s, dgmg_state* z, double t_next, const double* iapp,
                   const dgmg_pcg_opts* o, dgmg_pcg_stats* st, void* stream) {
    API_BEGIN
    (void)t_next;
    need_device(s);
    if (!z || !o || !st || !z->U || !z->Uprev || !z->W || !z->Wprev || !z->g) fail(DGMG_EINVAL, "null argument");
    hipStream_t hs = (hipStream_t)stream;
    RangeScope range(s, "dgmg time step");
    auto mark = [&](int k) {
        if (s->phase_on) HIPCHK(hipEventRecord(s->phase_ev[k], hs));
    };
    mark(0);
    // gates W_{n+1} into the W_{n-1} buffer, nodal ionic current g
    k_ionic<<<blocks_for(s->N), 256, 0, hs>>>(s->N, s->ip, z->U, z->Uprev, z->W, z->Wprev, z->Wprev, z->g);
    mark(1);
    // load vector; the warm start U_n is written into the U_{n-1} buffer
    const int cells_per = 256 / s->b;
    const unsigned nblk = (unsigned)((s->lv[0].n + cells_per - 1) / cells_per);
    DISPATCH_B(s->b, k_rhs<BV><<<nblk, cells_per * BV, 0, hs>>>(s->lv[0].n, s->ip, s->cU, s->mass, z->U,
                                                                 z->Uprev, iapp, z->g, s->bwork, z->Uprev));
    HIPCHK(hipGetLastError());
    mark(2);
    int rc = pcg(s, s->bwork, z->Uprev, *o, st, hs, s->partial, s->sc);
    mark(3);
    if (s->phase_on) ++s->phase_n;
    std::swap(z->U, z->Uprev);
    std::swap(z->W, z->Wprev);
    return rc;
    API_END
}

static void need_multi(const dgmg_solver* s, int32_t nrhs) {
    need_device(s);
    if (nrhs != DGMG_MULTI_RHS) fail(DGMG_EINVAL, "nrhs must be DGMG_MULTI_RHS");
    if (s->max_rhs < nrhs) fail(DGMG_EINVAL, "solver was set up with max_rhs < nrhs");
}

int dgmg_pcg_solve_multi(dgmg_solver* s, int32_t nrhs, const double* b, double* x, const dgmg_pcg_opts* o,
                         dgmg_pcg_stats* st, void* stream) {
    API_BEGIN
    need_multi(s, nrhs);
    if (!b || !x || !o || !st) fail(DGMG_EINVAL, "null argument");
    int rc = DGMG_OK;
    DISPATCH_R(nrhs, rc = pcg_multi<RV>(s, b, x, *o, st, (hipStream_t)stream));
    return rc;
    API_END
}

int dgmg_time_step_multi(dgmg_solver* s, int32_t nrhs, dgmg_state* z, double t_next, const double* iapp,
                         const dgmg_pcg_opts* o, dgmg_pcg_stats* st, void* stream) {
    API_BEGIN
    (void)t_next;
    need_multi(s, nrhs);
    if (!z || !o || !st || !z->U || !z->Uprev || !z->W || !z->Wprev || !z->g) fail(DGMG_EINVAL, "null argument");
    hipStream_t hs = (hipStream_t)stream;
    const int64_t NR = s->N * nrhs;
    // pointwise: the gates of all columns are one S x (N nrhs) array
    k_ionic<<<blocks_for(NR), 256, 0, hs>>>(NR, s->ip, z->U, z->Uprev, z->W, z->Wprev, z->Wprev, z->g);
    const int cells_per = 256 / s->b;
    const unsigned nblk = (unsigned)((s->lv[0].n + cells_per - 1) / cells_per);
    int rc = DGMG_OK;
    DISPATCH_R(nrhs, {
        DISPATCH_B(s->b, k_rhs_m<BV, RV><<<nblk, cells_per * BV, 0, hs>>>(
                             s->lv[0].n, s->ip, s->cU, s->mass, z->U, z->Uprev, iapp, z->g, s->bwork, z->Uprev));
        HIPCHK(hipGetLastError());
        rc = pcg_multi<RV>(s, s->bwork, z->Uprev, *o, st, hs);
    });
    std::swap(z->U, z->Uprev);
    std::swap(z->W, z->Wprev);
    return rc;
    API_END
}

int dgmg_apply_multi(dgmg_solver* s, int32_t level, int32_t prec, int32_t nrhs, const double* x, double* y,
                     void* stream) {
    API_BEGIN
    need_multi(s, nrhs);
    if (!x || !y) fail(DGMG_EINVAL, "null argument");
    if (level < 0 || level >= s->L) fail(DGMG_EINVAL, "level out of range");
    if (level == s->L - 1 && s->L > 1) fail(DGMG_EUNSUPPORTED, "the coarsest level is stored factorised");
    hipStream_t hs = (hipStream_t)stream;
    DevLevel& L = s->lv[level];
    const int64_t NR = L.N * nrhs;
    DISPATCH_R(nrhs, {
        if (prec == DGMG_PREC_FP64) {
            launch_apply<double, RV>(s, L, x, y, nullptr, nullptr, hs);
        } else {
            if (s->prec != DGMG_PREC_MIXED) fail(DGMG_EINVAL, "no FP32 copy in an FP64 solver");
            k_cast<double, float><<<blocks_for(NR), kWG, 0, hs>>>(NR, x, nullptr, (float*)L.vx2);
            launch_apply<float, RV>(s, L, (float*)L.vx2, (float*)L.vr, nullptr, nullptr, hs);
            k_cast<float, double><<<blocks_for(NR), kWG, 0, hs>>>(NR, (float*)L.vr, nullptr, y);
        }
    });
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_vcycle_multi(dgmg_solver* s, int32_t nrhs, const double* r, double* z, void* stream) {
    API_BEGIN
    need_multi(s, nrhs);
    if (!r || !z) fail(DGMG_EINVAL, "null argument");
    DISPATCH_R(nrhs, apply_vcycle<RV>(s, r, z, (hipStream_t)stream));
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_apply(dgmg_solver* s, int32_t level, int32_t prec, const double* x, double* y, void* stream) {
    API_BEGIN
    need_device(s);
    if (level < 0 || level >= s->L) fail(DGMG_EINVAL, "level out of range");
    hipStream_t hs = (hipStream_t)stream;
    DevLevel& L = s->lv[level];
    if (level == s->L - 1 && s->L > 1) fail(DGMG_EUNSUPPORTED, "the coarsest level is stored factorised");
    if (prec == DGMG_PREC_FP64) {
        launch_apply<double>(s, L, x, y, nullptr, nullptr, hs);
    } else {
        if (s->prec != DGMG_PREC_MIXED) fail(DGMG_EINVAL, "no FP32 copy in an FP64 solver");
        k_cast<double, float><<<blocks_for(L.N), kWG, 0, hs>>>(L.N, x, nullptr, (float*)L.vx2);
        launch_apply<float>(s, L, (float*)L.vx2, (float*)L.vr, nullptr, nullptr, hs);
        k_cast<float, double><<<blocks_for(L.N), kWG, 0, hs>>>(L.N, (float*)L.vr, nullptr, y);
    }
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_vcycle(dgmg_solver* s, const double* r, double* z, void* stream) {
    API_BEGIN
    need_device(s);
    if (!r || !z) fail(DGMG_EINVAL, "null argument");
    apply_vcycle(s, r, z, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_mass_apply(dgmg_solver* s, const double* f, double* b, void* stream) {
    API_BEGIN
    need_device(s);
    DISPATCH_B(s->b, k_mass<BV><<<blocks_for(s->N), 256, 0, (hipStream_t)stream>>>(s->lv[0].n, s->mass, f, b));
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_profile_begin(dgmg_solver* s, int32_t kind, int32_t level) {
    API_BEGIN
    need_device(s);
    if (kind < 0 || kind > PK_COARSE) fail(DGMG_EINVAL, "unknown kernel kind");
    s->prof_kind = kind;
    s->prof_level = level;
    s->prof_used = 0;
    return DGMG_OK;
    API_END
}

int dgmg_profile_end(dgmg_solver* s, int64_t* launches, double* total_ms) {
    API_BEGIN
    need_device(s);
    double tot = 0.0;
    for (size_t k = 0; k < s->prof_used; ++k) {
        HIPCHK(hipEventSynchronize(s->prof_ev[k].second));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, s->prof_ev[k].first, s->prof_ev[k].second));
        tot += ms;
    }
    if (launches) *launches = (int64_t)s->prof_used;
    if (total_ms) *total_ms = tot;
    s->prof_kind = -1;
    s->prof_level = -1;
    s->prof_used = 0;
    return DGMG_OK;
    API_END
}

int dgmg_set_phase_timing(dgmg_solver* s, int32_t on) {
    API_BEGIN
    need_device(s);
    if (on && !s->phase_ev[0])
        for (hipEvent_t& e : s->phase_ev) HIPCHK(hipEventCreate(&e));
    s->phase_on = on ? 1 : 0;
    s->phase_n = 0;
    return DGMG_OK;
    API_END
}

int dgmg_step_phase_ms(dgmg_solver* s, double* ms) {
    API_BEGIN
    need_device(s);
    if (!ms) fail(DGMG_EINVAL, "null argument");
    if (!s->phase_on || s->phase_n == 0) fail(DGMG_EINVAL, "no time step was timed since phase timing was switched on");
    HIPCHK(hipEventSynchronize(s->phase_ev[3]));
    for (int k = 0; k < 3; ++k) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, s->phase_ev[k], s->phase_ev[k + 1]));
        ms[k] = t;
    }
    return DGMG_OK;
    API_END
}

int dgmg_set_sensors(dgmg_solver* s, int32_t n, const int64_t* cells, const double* ref) {
    API_BEGIN
    need_device(s);
    if (n < 0 || (n > 0 && (!cells || !ref))) fail(DGMG_EINVAL, "bad sensor arrays");
    RefElement re;
    re.init(s->dim, s->p);
    std::vector<int64_t> c(cells, cells + n);
    std::vector<double> w((size_t)n * s->b);
    for (int k = 0; k < n; ++k) {
        if (c[k] < 0 || c[k] >= s->lv[0].n) fail(DGMG_EINVAL, "sensor cell out of range");
        tensor_eval(re, ref + (size_t)k * s->dim, &w[(size_t)k * s->b], nullptr);
    }
    s->scell = s->upload(c);
    s->sw = s->upload(w);
    s->n_sensors = n;
    return DGMG_OK;
    API_END
}

int dgmg_sensor_misfit(dgmg_solver* s, const double* U, const double* target, double* Ubar,
                       double* loss, void* stream) {
    API_BEGIN
    need_device(s);
    if (!U || !target || !loss) fail(DGMG_EINVAL, "null argument");
    DISPATCH_B(s->b, k_sensor_misfit<BV><<<1, 256, 0, (hipStream_t)stream>>>(s->n_sensors, s->scell, s->sw, U,
                                                                              target, Ubar, loss));
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_adjoint_step(dgmg_solver* s, const double* U, const double* Uprev, const double* W,
                      const double* Wprev, const double* lambda, const double* Wbar_in, double* Ubar,
                      double* Uprevbar, double* Wbar, double* Wprevbar, void* stream) {
    API_BEGIN
    need_device(s);
    if (!s->has_adjoint) fail(DGMG_EINVAL, "solver was set up without adjoint data");
    if (!U || !Uprev || !W || !Wprev || !lambda || !Wbar_in || !Ubar || !Uprevbar || !Wbar || !Wprevbar)
        fail(DGMG_EINVAL, "null argument");
    const int cells_per = 256 / s->b;
    const unsigned nblk = (unsigned)((s->lv[0].n + cells_per - 1) / cells_per);
    DISPATCH_B(s->b, k_adjoint_step<BV><<<nblk, cells_per * BV, 0, (hipStream_t)stream>>>(
                         s->lv[0].n, s->ip, s->cU, s->mass, U, Uprev, W, Wprev, lambda, Wbar_in, Ubar,
                         Uprevbar, Wbar, Wprevbar));
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_grad_accumulate(dgmg_solver* s, const double* lambda, const double* U, double* grad,
                         void* stream) {
    API_BEGIN
    need_device(s);
    if (!s->has_adjoint) fail(DGMG_EINVAL, "solver was set up without adjoint data");
    if (!lambda || !U || !grad) fail(DGMG_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const int b = s->b;
    const int fpw = 256 / (2 * b), cpw = 256 / b;
    DISPATCH_B(b, k_grad_faces<BV><<<(unsigned)((s->nf0 + fpw - 1) / fpw), 256, 0, st>>>(
                      (int32_t)s->nf0, s->adj_fc, s->adjX, lambda, U, s->adjq));
    DISPATCH_B(b, k_grad_cells<BV><<<(unsigned)((s->lv[0].n + cpw - 1) / cpw), 256, 0, st>>>(
                      s->lv[0].n, s->adjS, s->adj_nptr, s->adj_ncode, s->adjq, lambda, U, grad));
    HIPCHK(hipGetLastError());
    return DGMG_OK;
    API_END
}

int dgmg_kernel_bench(dgmg_solver* s, int32_t kind, int32_t level, int32_t nrhs, int32_t reps, void* stream,
                      double* avg_ms) {
    API_BEGIN
    need_device(s);
    if (level < 0 || level >= s->L - 1 || reps < 1) fail(DGMG_EINVAL, "bad level or repetition count");
    if (kind != PK_CHEB_STEP && kind != PK_RESIDUAL) fail(DGMG_EINVAL, "kernel kind not benchmarkable");
    if (nrhs != 1) need_multi(s, nrhs);
    hipStream_t st = (hipStream_t)stream;
    DevLevel& L = s->lv[level];
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    auto run = [&](auto tag, auto rtag) {
        using T = decltype(tag);
        constexpr int R = decltype(rtag)::value;
        const int64_t NR = L.N * R;
        T *x = (T*)L.vx, *r = (T*)L.vr, *d = (T*)L.vd, *d2 = (T*)L.vd2, *x2 = (T*)L.vx2;
        const T* bb = (const T*)L.vb;
        // the kernel the solver runs: with the cells' block inverses when set
        const T* bjk = (R == 1 && s->jacobi == DGMG_JACOBI_CELL_BLOCK) ? BJof<T>(L) : nullptr;
        // defined inputs
        k_fill<T><<<blocks_for(NR), kWG, 0, st>>>(NR, x, (T)1e-3);
        k_fill<T><<<blocks_for(NR), kWG, 0, st>>>(NR, d, (T)1e-3);
        k_fill<T><<<blocks_for(NR), kWG, 0, st>>>(NR, r, (T)1e-3);
        HIPCHK(hipEventRecord(a, st));
        for (int k = 0; k < reps; ++k) {
            if (kind == PK_CHEB_STEP) {
                launch_step<T, R>(s, L, d, x, r, d2, (T)0.5, (T)0.1, 0, 0, st, bjk);
                std::swap(d, d2);
            } else {
                launch_residual<T, R>(s, L, x, d, bb ? bb : r, r, d2, (T)0.5, x2, nullptr, st, nullptr,
                                      nullptr, nullptr, bjk);
            }
        }
        HIPCHK(hipEventRecord(b, st));
    };
    using R1 = std::integral_constant<int, 1>;
    using R8 = std::integral_constant<int, DGMG_MULTI_RHS>;
    if (s->prec == DGMG_PREC_MIXED) {
        if (nrhs == 1) run(float{}, R1{});
        else run(float{}, R8{});
    } else {
        if (nrhs == 1) run(double{}, R1{});
        else run(double{}, R8{});
    }
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / reps;
    return DGMG_OK;
    API_END
}

int dgmg_export_level(const dgmg_solver* s, int32_t level, double* diag, int64_t* fc, double* fb,
                      double* P, int64_t* parents) {
    API_BEGIN
    if (!s) fail(DGMG_EINVAL, "null solver");
    if (level < 0 || level >= s->L) fail(DGMG_EINVAL, "level out of range");
    const BlockOp& A = s->ops[level];
    if (diag) std::copy(A.diag.begin(), A.diag.end(), diag);
    if (fc) std::copy(A.fc.begin(), A.fc.end(), fc);
    if (fb) std::copy(A.fblk.begin(), A.fblk.end(), fb);
    if (level + 1 < s->L) {
        if (P) std::copy(s->Ph[level].begin(), s->Ph[level].end(), P);
        if (parents) std::copy(s->parents[level].begin(), s->parents[level].end(), parents);
    }
    return DGMG_OK;
    API_END
}

}  // extern "C"
