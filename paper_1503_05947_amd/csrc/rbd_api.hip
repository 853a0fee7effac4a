// Host side of the RBD library: argument validation, workspace layout,
// launch plans and the C ABI declared in include/rbd.h.
//
// rbd_fit enqueues the whole greedy loop on the caller's stream without ever
// waiting for the device: for step s = 0 .. D-1 it launches the kernels of
// one step with d = s (the device keeps the real d, and every kernel returns
// at once after the stop flag is set).  The host therefore knows an upper
// bound of d for each launch and sizes register tiles (KC) from it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/rbd.h"
#include "rbd_kernels.h"
#include "rbd_loop.h"
#include "rbd_proj.h"

namespace {

using namespace rbd;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int elem_bytes(rbd_dtype t) {
    switch (t) {
        case RBD_F32: return 4;
        case RBD_BF16: return 2;
        case RBD_F16: return 2;
        case RBD_F64: return 8;
    }
    return 0;
}
int vec_elems(rbd_dtype t) { return 16 / elem_bytes(t); }

struct FitPlan {
    int64_t m = 0, n = 0;
    int D = 0, d_max = 0;
    rbd_dtype xt = RBD_F32;
    // X-scan
    int sc_tpb = 256, sc_ch = 1, sc_tiles = 1, sc_rows = 0, sc_S = 0;
    // update (combine partials, downdate, argmax)
    int up_ncb = 0, up_SG = 1;
    // Gram-Schmidt passes
    int cg_rows = 0, cg_S = 0, cg_group = 32, cg_ngroups = 0;
    // exact residual evaluation
    int rc_rows = 0, rc_S = 0, rc_grid = 0, rf_grid = 0;
    int ntickets = 0;
    // persistent loop (A = I, cache-resident X): workgroups, Gram-Schmidt
    // workgroups, rows per Gram-Schmidt workgroup, columns per workgroup
    bool loop = false;
    bool y32 = false;           // the basis is kept in FP32 (o_yf) and copied out at the end
    size_t o_yf = 0;
    int64_t ldyf = 0;           // its leading dimension: d_max rounded up to even (8-byte column pairs)
    int lp_G = 0, lp_Gc = 0, lp_RB = 0, lp_CW = 0;
    size_t o_lp_bv = 0, o_lp_bi = 0, o_lp_bc = 0, o_lp_part = 0, o_lp_qc = 0, o_lp_ql = 0, o_lp_rp = 0;
    // workspace offsets (bytes)
    int ntiles = 0;
    size_t o_state, o_tickets, o_e2, o_base2, o_flist, o_bres_v, o_bres_i, o_v1, o_v2, o_h2, o_nu2, o_g, o_xp, o_M, o_mh, o_hw, o_ys,
        o_part,
        o_l2, o_rpart, total;
};

// The persistent loop (rbd_loop.h) runs the whole fit in one launch when X is
// small enough to stay in the caches from step to step; larger X streams from
// HBM with one launch per kernel of a step.  RBD_LOOP=0 in the environment
// turns the persistent loop off, RBD_LOOP=1 uses it whenever the shape allows,
// RBD_LOOP_G sets its workgroup count (both for measurements); the workgroup
// count assumes the MI355X's 256 CUs and is checked against the device at
// launch.
constexpr double kLoopMaxBytes = 64.0 * 1024 * 1024;
void plan_loop(FitPlan* P) {
    P->loop = false;
    const char* env = std::getenv("RBD_LOOP");
    const int force = env ? std::atoi(env) : -1;
    if (force == 0) return;
    const double bytes = (double)P->m * (double)P->n * elem_bytes(P->xt);
    if (force != 1 && bytes > kLoopMaxBytes) return;
    if (P->m >= ((int64_t)1 << 30) || P->n >= ((int64_t)1 << 30)) return;
    // one workgroup per 128 KB of X, a multiple of 8 (whole XCDs), 32 .. 256
    // (measured on the 2048 x 2048 FP32 field: 32, 64, 128, 256 workgroups take
    // 32.8, 28.2, 27.0, 29.5 us per fixed step; on the 512 x 256 one, 8, 16, 32,
    // 64 workgroups take 31.1, 26.2, 23.5, 22.9 us per step: the exact refreshes
    // are split over all of them)
    int64_t G = (int64_t)(bytes / (128.0 * 1024));
    G = std::max<int64_t>(32, std::min<int64_t>(kLoopMaxG, cdiv(std::max<int64_t>(G, 1), 8) * 8));
    // at most kLoopMaxCW columns and kLoopMaxRB Gram-Schmidt rows per workgroup;
    // up to 32 Gram-Schmidt workgroups of at least 64 rows
    const int64_t Gc = std::max<int64_t>(cdiv(P->m, kLoopMaxRB), std::min<int64_t>(32, cdiv(P->m, 64)));
    G = std::max<int64_t>(G, cdiv(cdiv(P->n, kLoopMaxCW), 8) * 8);
    G = std::max<int64_t>(G, cdiv(Gc, 8) * 8);
    if (const char* g_env = std::getenv("RBD_LOOP_G")) {      // measurement override, a multiple of 8
        const int64_t g = std::atoll(g_env);
        if (g >= 8 && g % 8 == 0) G = std::max<int64_t>(g, cdiv(Gc, 8) * 8);
    }
    if (G > kLoopMaxG) return;
    const int64_t RB = cdiv(P->m, Gc);
    int CW = 1;
    while ((int64_t)CW * G < P->n) CW <<= 1;
    if (CW > kLoopMaxCW || RB > kLoopMaxRB) return;
    P->loop = true;
    P->lp_G = (int)G;
    P->lp_Gc = (int)Gc;
    P->lp_RB = (int)RB;
    P->lp_CW = CW;
}

bool make_fit_plan(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, FitPlan* P, int basis = RBD_BASIS_F64) {
    if (m < 1 || n < 1 || d_max < 1) return false;
    if (basis != RBD_BASIS_F64 && basis != RBD_BASIS_F32) return false;
    P->y32 = (basis == RBD_BASIS_F32);
    if (elem_bytes(xt) == 0) return false;
    if (n >= (int64_t)INT32_MAX || m >= ((int64_t)1 << 40)) return false;
    P->m = m;
    P->n = n;
    P->xt = xt;
    P->d_max = d_max;
    P->D = (int)std::min<int64_t>(d_max, std::min(m, n));
    if (P->D > RBD_MAX_D) return false;

    // X-scan: 16-byte loads.  Long-lived workgroups stream best (measured on
    // MI355X at 1048576 x 4096: 512-1024 workgroups of 2048-row slabs reach
    // 99% of a plain read stream).  4- and 8-byte types give each thread up to
    // 4 column chunks so a workgroup covers whole rows; 2-byte types keep one
    // chunk and 8 rows in flight instead.
    const int N = vec_elems(xt);
    const int64_t nvec = cdiv(n, N);
    P->sc_tpb = nvec >= 256 ? 256 : (nvec >= 128 ? 128 : 64);
    const bool narrow = elem_bytes(xt) == 2;
    P->sc_ch = narrow ? 1 : (nvec >= 4 * 256 ? 4 : (nvec >= 2 * 256 ? 2 : 1));
    P->sc_tiles = (int)cdiv(nvec, (int64_t)P->sc_tpb * P->sc_ch);
    const int64_t target_wg = narrow ? 1024 : 512;
    int64_t rows = cdiv(m * P->sc_tiles, target_wg);
    rows = std::max<int64_t>(16, std::min<int64_t>(rows, 4096));
    P->sc_rows = (int)rows;
    P->sc_S = (int)cdiv(m, rows);

    P->up_ncb = (int)cdiv(n, 256);
    P->up_SG = (int)std::max<int64_t>(1, std::min<int64_t>(64, cdiv(P->sc_S, 16)));

    // Gram-Schmidt: 4 waves per block, ~2048 blocks, rows a multiple of 16
    int64_t crow = cdiv(m, 2048);
    crow = std::max<int64_t>(16, cdiv(crow, 16) * 16);
    P->cg_rows = (int)crow;
    P->cg_S = (int)cdiv(m, crow);
    P->cg_group = 32;
    P->cg_ngroups = (int)cdiv(P->cg_S, P->cg_group);

    // exact residuals: 64-column tiles of the queue, at most 256 row slabs of a multiple of 128 rows
    P->ntiles = (int)cdiv(n, 64);
    int64_t rrow = std::max<int64_t>(128, cdiv(cdiv(m, 256), 128) * 128);
    P->rc_rows = (int)std::min<int64_t>(rrow, INT32_MAX / 2);
    P->rc_S = (int)cdiv(m, rrow);
    P->rc_grid = (int)std::min<int64_t>(2048, (int64_t)P->ntiles * P->rc_S);
    P->rf_grid = (int)cdiv(n, 256);

    P->ntickets = (int)std::max<int64_t>(P->up_ncb + 1, P->cg_ngroups + 1) + 8;
    plan_loop(P);            // inputs the persistent loop takes keep the FP64 basis in every mode

    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    P->o_state = take(sizeof(State));
    P->o_tickets = take(sizeof(unsigned) * P->ntickets);
    P->o_e2 = take(8 * n);
    P->o_base2 = take(8 * n);
    P->o_flist = take(4 * n);
    P->o_bres_v = take(8 * P->up_ncb);
    P->o_bres_i = take(8 * P->up_ncb);
    P->o_v1 = take(8 * m);
    P->o_v2 = take(8 * m);
    P->o_h2 = take(8 * 2 * ((size_t)RBD_MAX_D + 1));   // two h2 buffers (lagged path: this step and the last)
    P->o_nu2 = take(8);
    P->o_g = take(8 * m);
    P->o_xp = take(8 * m);
    P->o_M = take(8 * (size_t)std::max(P->D, 1) * std::max(P->D, 1));    // Y'WY (diagonal A)
    P->o_mh = take(8 * ((size_t)RBD_MAX_D + 1));
    P->o_hw = take(8 * (size_t)RBD_MAX_D);
    P->o_ys = take(8 * 8 * (size_t)m);      // staged basis columns (every path), m x 8 column-major
    // scan partials (two rows of n per slab with an A-norm); Gram-Schmidt partials.  The
    // lagged path (rows of n) and the SPD path (rows of 2n) add up to ceil(D / kTcorr)
    // correction rows after the scan's slabs.
    const size_t kp_max = (size_t)cdiv(std::max(P->D, 1), kTcorr);
    const size_t part_elems = std::max<size_t>(((size_t)P->sc_S + kp_max) * 2 * n,
                                               (size_t)P->cg_S * 2 * (std::max(P->D, 1) + 1));
    P->o_part = take(8 * part_elems);
    const size_t l2_elems =
        std::max<size_t>(((size_t)P->up_SG + kp_max + 1) * 2 * n, (size_t)P->cg_ngroups * std::max(P->D, 1));
    P->o_l2 = take(8 * l2_elems);
    P->o_rpart = take(8 * (size_t)P->rc_S * n);
    if (P->y32) {
        P->ldyf = d_max + (d_max & 1);
        P->o_yf = take(4 * (size_t)m * P->ldyf);
    }
    if (P->loop) {
        P->o_lp_bv = take(8 * 2 * (size_t)P->lp_G);
        P->o_lp_bi = take(8 * 2 * (size_t)P->lp_G);
        P->o_lp_bc = take(8 * 2 * (size_t)P->lp_G);
        P->o_lp_part = take(8 * (size_t)P->lp_Gc * (P->D + 1));
        P->o_lp_qc = take(4 * (size_t)P->lp_G);
        P->o_lp_ql = take(4 * (size_t)P->lp_G * P->lp_CW);
        P->o_lp_rp = take(8 * (size_t)P->lp_G * n);
    }
    P->total = o;
    return true;
}

// Compute units of the current device (cached per device).
int device_cus() {
    static std::mutex mu;
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        cus[dev] = v;
    }
    return cus[dev];
}

// Passes over Y(:, 0:d) use non-temporal loads once that read exceeds the
// last-level cache (256 MB): measured on MI355X, a 4 GB row-major Y streams
// at 6.3 TB/s with ordinary loads and 6.9-7.0 TB/s with non-temporal ones.
bool y_stream(const FitPlan& P, int d) { return (double)P.m * (double)d * 8.0 > 256.0 * 1024 * 1024; }

int kc_for(int d) {
    const int need = std::max(1, (d + kWave - 1) / kWave);
    int kc = 1;
    while (kc < need) kc <<= 1;
    return kc;
}

// ---------------------------------------------------------------------------
// optional HIP-event phase profiler (per host thread)
// ---------------------------------------------------------------------------
struct Profiler {
    bool on = false;
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Mark { int phase; size_t a, b; };
    std::vector<Mark> marks;
    size_t fit_start = 0;
    std::vector<size_t> steps;      // event index at the end of each step of the current fit
    bool failed = false;

    hipEvent_t* take(hipStream_t s) {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { failed = true; return nullptr; }
            pool.push_back(e);
        }
        hipEvent_t* e = &pool[used];
        if (hipEventRecord(*e, s) != hipSuccess) failed = true;
        ++used;
        return e;
    }
};
thread_local Profiler g_prof;
thread_local size_t g_prof_open = 0;

inline void prof_fit_begin(hipStream_t s) {
    if (!g_prof.on) return;
    g_prof.steps.clear();
    g_prof.fit_start = g_prof.used;
    g_prof.take(s);
}
inline void prof_begin(int phase, hipStream_t s) {
    if (!g_prof.on || !(g_prof.mask & (1u << phase))) return;
    g_prof_open = g_prof.used;
    g_prof.take(s);
}
inline void prof_end(int phase, hipStream_t s) {
    if (!g_prof.on || !(g_prof.mask & (1u << phase))) return;
    const size_t b = g_prof.used;
    g_prof.take(s);
    g_prof.marks.push_back({phase, g_prof_open, b});
}
inline void prof_step(hipStream_t s) {
    if (!g_prof.on) return;
    g_prof.steps.push_back(g_prof.used);
    g_prof.take(s);
}

#define RBD_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return RBD_EDEVICE; \
    } while (0)

// X-scan launch for one plan: CH column chunks per thread (4/8-byte types),
// or one chunk with 8 rows in flight (2-byte types).
template <typename Tx, int MODE>
void launch_xscan(const FitPlan& P, const Tx* X, int64_t ldx, const double* v2, State* st, double* Y, int dcol,
                  double* part, int vec_ok, bool nt, hipStream_t s, const double* g2 = nullptr) {
    const dim3 grid(P.sc_tiles, P.sc_S);
    const size_t lds = MODE == kScanSqr ? 0 : sizeof(double) * P.sc_rows * (MODE == kScanDot2 ? 2 : 1);
#define RBD_XSCAN(U, NT, CH)                                                                                 \
    xscan_kernel<Tx, MODE, U, NT, CH><<<grid, P.sc_tpb, lds, s>>>(X, ldx, P.m, P.n, v2, st, Y, P.d_max, dcol, \
                                                                  P.sc_rows, part, vec_ok, g2)
    if (sizeof(Tx) == 2) {
        if (nt) RBD_XSCAN(8, true, 1);
        else RBD_XSCAN(8, false, 1);
    } else if (P.sc_ch == 4) {
        if (nt) RBD_XSCAN(4, true, 4);
        else RBD_XSCAN(4, false, 4);
    } else if (P.sc_ch == 2) {
        if (nt) RBD_XSCAN(4, true, 2);
        else RBD_XSCAN(4, false, 2);
    } else {
        if (nt) RBD_XSCAN(4, true, 1);
        else RBD_XSCAN(4, false, 1);
    }
#undef RBD_XSCAN
}

// Rows of Y in flight per wave: short rows (small d) are latency-bound, so keep
// more of them in flight; long rows are limited by registers.
constexpr int rows_in_flight(int KC) { return KC <= 2 ? 8 : (KC <= 8 ? 4 : 2); }

template <int KC>
void launch_cgs1(const FitPlan& P, const double* xp, const double* Y, const double* T, State* st, int d,
                 const double* ys, double* v1, double* part, hipStream_t s) {
    if (y_stream(P, d))
        cgs1_kernel<KC, rows_in_flight(KC), true><<<P.cg_S, 256, 0, s>>>(xp, P.m, Y, P.d_max, T, P.n, st, d,
                                                                          P.cg_rows, ys, v1, part, std::max(P.D, 1));
    else
        cgs1_kernel<KC, rows_in_flight(KC), false><<<P.cg_S, 256, 0, s>>>(xp, P.m, Y, P.d_max, T, P.n, st, d,
                                                                           P.cg_rows, ys, v1, part, std::max(P.D, 1));
}

template <int KC>
void launch_cgs1w(const FitPlan& P, const double* xp, const double* Y, const double* T, State* st, int d,
                  const double* w, const double* ys, double* v1, double* part, hipStream_t s) {
    if (y_stream(P, d))
        cgs1w_kernel<KC, rows_in_flight(KC), true><<<P.cg_S, 256, 0, s>>>(xp, P.m, Y, P.d_max, T, P.n, st, d,
                                                                           P.cg_rows, w, ys, v1, part, std::max(P.D, 1));
    else
        cgs1w_kernel<KC, rows_in_flight(KC), false><<<P.cg_S, 256, 0, s>>>(xp, P.m, Y, P.d_max, T, P.n, st, d,
                                                                            P.cg_rows, w, ys, v1, part, std::max(P.D, 1));
}

template <int KC>
void launch_gvec2(const FitPlan& P, double* Y, const State* st, int d, const double* v1, const double* h2,
                  const double* hw, const double* w, double* ys, double* v2, double* g, hipStream_t s) {
    if (y_stream(P, d))
        gvec2_kernel<KC, rows_in_flight(KC), true><<<P.cg_S, 256, 0, s>>>(Y, P.d_max, P.m, st, d, P.cg_rows, v1, h2,
                                                                           hw, w, ys, v2, g);
    else
        gvec2_kernel<KC, rows_in_flight(KC), false><<<P.cg_S, 256, 0, s>>>(Y, P.d_max, P.m, st, d, P.cg_rows, v1, h2,
                                                                            hw, w, ys, v2, g);
}

// rbd_fit_basis(RBD_BASIS_F32): steps below this column run on the FP64 basis
// (a multiple of 128, so the switch falls on a block boundary).
constexpr int kY32Switch = 128;

// The FP32-basis passes: two columns per lane, KC / 2 chunks of 128 columns.
constexpr int kc2_of(int KC) { return KC <= 2 ? 1 : KC / 2; }
constexpr int rows32(int KC) { return kc2_of(KC) <= 2 ? 8 : (kc2_of(KC) <= 4 ? 4 : 2); }

// The FP64-basis pass reads x_p from X itself; the FP32-basis pass reads the
// column gathered into xp (reading X there measured slower).
template <int KC, typename Tb, typename Tx>
void launch_cgs1_lag(const FitPlan& P, const Tx* X, int64_t ldx, const double* xp, Tb* Y, const double* T, State* st,
                     int d, const double* v1p, const double* h2p, double* v1, double* ys, double* part,
                     hipStream_t s) {
    if constexpr (std::is_same<Tb, float>::value) {
        constexpr int K2 = kc2_of(KC), R2 = rows32(KC);
        if (y_stream(P, d))
            cgs1_lag32_kernel<K2, R2, true><<<P.cg_S, 256, 0, s>>>(xp, P.m, Y, P.ldyf, T, P.n, st, d, P.cg_rows, v1p,
                                                                    h2p, v1, ys, part, std::max(P.D, 1));
        else
            cgs1_lag32_kernel<K2, R2, false><<<P.cg_S, 256, 0, s>>>(xp, P.m, Y, P.ldyf, T, P.n, st, d, P.cg_rows, v1p,
                                                                     h2p, v1, ys, part, std::max(P.D, 1));
    } else if (y_stream(P, d)) {
        cgs1_lag_kernel<KC, rows_in_flight(KC), true, Tb, Tx><<<P.cg_S, 256, 0, s>>>(X, ldx, P.m, Y, P.d_max, T, P.n, st, d,
                                                                              P.cg_rows, v1p, h2p, v1, ys, part,
                                                                              std::max(P.D, 1));
    } else {
        cgs1_lag_kernel<KC, rows_in_flight(KC), false, Tb, Tx><<<P.cg_S, 256, 0, s>>>(X, ldx, P.m, Y, P.d_max, T, P.n, st, d,
                                                                               P.cg_rows, v1p, h2p, v1, ys, part,
                                                                               std::max(P.D, 1));
    }
}

template <typename Tx>
void launch_gather(const FitPlan& P, const Tx* X, int64_t ldx, const State* st, double* xp, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(16384, cdiv(P.m, 256));
    gather_col_kernel<Tx><<<g, 256, 0, s>>>(X, ldx, P.m, st, xp);
}

template <int KC, bool FINAL, typename Tb>
void launch_ycol(const FitPlan& P, Tb* Y, const State* st, int d, const double* v1a, const double* v1b,
                 const double* h2a, const double* h2b, const double* ys, hipStream_t s) {
    if constexpr (std::is_same<Tb, float>::value) {
        constexpr int K2 = kc2_of(KC), R2 = rows32(KC);
        if (y_stream(P, FINAL ? P.D : d))
            ycol32_kernel<K2, R2, FINAL, true><<<P.cg_S, 256, 0, s>>>(Y, P.ldyf, P.m, st, d, P.cg_rows, v1a, v1b,
                                                                       h2a, h2b, ys);
        else
            ycol32_kernel<K2, R2, FINAL, false><<<P.cg_S, 256, 0, s>>>(Y, P.ldyf, P.m, st, d, P.cg_rows, v1a, v1b,
                                                                        h2a, h2b, ys);
    } else if (y_stream(P, FINAL ? P.D : d)) {
        // FINAL: the column index is only known on the device; size the choice by D
        ycol_kernel<KC, rows_in_flight(KC), FINAL, true, Tb><<<P.cg_S, 256, 0, s>>>(Y, P.d_max, P.m, st, d, P.cg_rows,
                                                                                 v1a, v1b, h2a, h2b, ys);
    } else {
        ycol_kernel<KC, rows_in_flight(KC), FINAL, false, Tb><<<P.cg_S, 256, 0, s>>>(Y, P.d_max, P.m, st, d, P.cg_rows,
                                                                                  v1a, v1b, h2a, h2b, ys);
    }
}

template <bool FINAL, typename Tb>
void launch_ycol_kc(int kc, const FitPlan& P, Tb* Y, const State* st, int d, const double* v1a,
                    const double* v1b, const double* h2a, const double* h2b, const double* ys, hipStream_t s) {
    switch (kc) {
        case 1: launch_ycol<1, FINAL, Tb>(P, Y, st, d, v1a, v1b, h2a, h2b, ys, s); break;
        case 2: launch_ycol<2, FINAL, Tb>(P, Y, st, d, v1a, v1b, h2a, h2b, ys, s); break;
        case 4: launch_ycol<4, FINAL, Tb>(P, Y, st, d, v1a, v1b, h2a, h2b, ys, s); break;
        case 8: launch_ycol<8, FINAL, Tb>(P, Y, st, d, v1a, v1b, h2a, h2b, ys, s); break;
        default: launch_ycol<16, FINAL, Tb>(P, Y, st, d, v1a, v1b, h2a, h2b, ys, s); break;
    }
}

template <int KC>
void launch_cgs2u(const FitPlan& P, double* Y, const State* st, int d, const double* v1, const double* h2,
                  const double* u, double* ys, double* v2, double* part, hipStream_t s) {
    if (y_stream(P, d))
        cgs2u_kernel<KC, rows_in_flight(KC), true><<<P.cg_S, 256, 0, s>>>(Y, P.d_max, P.m, st, d, P.cg_rows, v1, h2,
                                                                           u, ys, v2, part, std::max(P.D, 1));
    else
        cgs2u_kernel<KC, rows_in_flight(KC), false><<<P.cg_S, 256, 0, s>>>(Y, P.d_max, P.m, st, d, P.cg_rows, v1,
                                                                            h2, u, ys, v2, part, std::max(P.D, 1));
}

// the staged basis columns into Y (before an exact refresh: FINAL = false, cols = d + 1)
template <bool FINAL>
void launch_ys_flush(const FitPlan& P, double* Y, const State* st, int cols, const double* ys, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(8192, cdiv(P.m * 8, 256));
    ys_flush_kernel<FINAL><<<g, 256, 0, s>>>(Y, P.d_max, P.m, st, cols, ys);
}

// out[c] = sum_r part[r * ldp + c] for c < len in a fixed order: rows in groups
// of `per`, then the group sums, through `l2` (ceil(rows/per) x ldp); with at
// most 256 rows, one sequential level.
void launch_sum_rows(const State* st, const double* part, int64_t ldp, int rows, int per, int64_t len, double* l2,
                     double* out, int64_t ldo_final, hipStream_t s) {
    const unsigned gx = (unsigned)cdiv(len, 256);
    if (rows <= 256) {          // few rows: one level, one launch
        reduce_rows_kernel<<<dim3(gx, 1), 256, 0, s>>>(st, part, ldp, rows, rows, len, out, ldo_final);
        return;
    }
    const int groups = (int)cdiv(rows, per);
    reduce_rows_kernel<<<dim3(gx, groups), 256, 0, s>>>(st, part, ldp, rows, per, len, l2, ldp);
    reduce_rows_kernel<<<dim3(gx, 1), 256, 0, s>>>(st, l2, ldp, groups, groups, len, out, ldo_final);
}

template <typename Tx>
int fit_typed(const FitPlan& P, const Tx* X, int64_t ldx, double tol, int rel, int64_t start, double* Y,
              double* T, int64_t* pivots, double* col_err, double* err_hist, int32_t* d_out, int32_t* status,
              int32_t* stop_reason, char* ws, hipStream_t s, const double* w) {
    State* st = reinterpret_cast<State*>(ws + P.o_state);
    unsigned* tickets = reinterpret_cast<unsigned*>(ws + P.o_tickets);
    double* e2 = reinterpret_cast<double*>(ws + P.o_e2);
    double* base2 = reinterpret_cast<double*>(ws + P.o_base2);
    int* flist = reinterpret_cast<int*>(ws + P.o_flist);
    double* bres_v = reinterpret_cast<double*>(ws + P.o_bres_v);
    int64_t* bres_i = reinterpret_cast<int64_t*>(ws + P.o_bres_i);
    double* v1 = reinterpret_cast<double*>(ws + P.o_v1);
    double* v2 = reinterpret_cast<double*>(ws + P.o_v2);
    double* h2 = reinterpret_cast<double*>(ws + P.o_h2);
    double* part = reinterpret_cast<double*>(ws + P.o_part);
    double* l2 = reinterpret_cast<double*>(ws + P.o_l2);
    double* rpart = reinterpret_cast<double*>(ws + P.o_rpart);
    double* g = reinterpret_cast<double*>(ws + P.o_g);
    double* hw = reinterpret_cast<double*>(ws + P.o_hw);
    double* xp = reinterpret_cast<double*>(ws + P.o_xp);
    double* Mw = reinterpret_cast<double*>(ws + P.o_M);
    double* mh = reinterpret_cast<double*>(ws + P.o_mh);
    double* ys = reinterpret_cast<double*>(ws + P.o_ys);
    const bool W = (w != nullptr);
    const int64_t nw = W ? 2 * P.n : P.n;     // scan partial row length

    const int N = Ld<Tx>::N;
    const int vec_ok = (ldx % N == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    const bool nt = (double)P.m * (double)ldx * sizeof(Tx) > 512.0 * 1024 * 1024;

    prof_fit_begin(s);
    init_state_kernel<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(P.ntickets, 256))), 256, 0, s>>>(st, tickets,
                                                                                              P.ntickets, P.D);
    RBD_LAUNCH_CHECK();
    if (!W && P.loop && P.lp_G <= device_cus()) {
        // the whole loop in one launch; the last two tickets (zeroed above)
        // are its barrier counter and abort flag
        LoopWs lw;
        lw.bar = tickets + P.ntickets - 2;
        lw.abort_flag = reinterpret_cast<int*>(tickets + P.ntickets - 1);
        lw.part = reinterpret_cast<double*>(ws + P.o_lp_part);
        lw.v1 = v1;
        lw.bval = reinterpret_cast<double*>(ws + P.o_lp_bv);
        lw.bidx = reinterpret_cast<int64_t*>(ws + P.o_lp_bi);
        lw.bcnt = reinterpret_cast<double*>(ws + P.o_lp_bc);
        lw.qcnt = reinterpret_cast<int*>(ws + P.o_lp_qc);
        lw.qlist = reinterpret_cast<int*>(ws + P.o_lp_ql);
        lw.rpart = reinterpret_cast<double*>(ws + P.o_lp_rp);
        LoopOut lo{Y, T, pivots, col_err, err_hist, d_out, status, stop_reason};
        prof_begin(RBD_PHASE_LOOP, s);
        loop_kernel<Tx><<<P.lp_G, kLoopThreads, 0, s>>>(X, ldx, (int)P.m, (int)P.n, P.D, P.d_max, tol, rel, start, lo,
                                                        lw, P.lp_Gc, P.lp_RB, P.lp_CW, vec_ok);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_LOOP, s);
        return RBD_OK;
    }
    // pre-computation of diag(X'X) (section 3.3): e_j^2 = ||x_j||^2, E_0, first column
    prof_begin(RBD_PHASE_COLNORM, s);
    if (W) launch_xscan<Tx, kScanSqrW>(P, X, ldx, w, st, Y, 0, part, vec_ok, nt, s);
    else launch_xscan<Tx, kScanSqr>(P, X, ldx, nullptr, st, Y, 0, part, vec_ok, nt, s);
    RBD_LAUNCH_CHECK();
    prof_end(RBD_PHASE_COLNORM, s);
    prof_begin(RBD_PHASE_INIT, s);
    const int up_per = (int)cdiv(P.sc_S, P.up_SG);
    const dim3 red_grid((unsigned)cdiv(P.n, 256), (unsigned)cdiv(P.sc_S, up_per));
    const dim3 red_grid_step((unsigned)cdiv(nw, 256), (unsigned)cdiv(P.sc_S, up_per));
    const int up_groups = (int)cdiv(P.sc_S, up_per);
    reduce_rows_kernel<<<red_grid, 256, 0, s>>>(nullptr, part, P.n, P.sc_S, up_per, P.n, l2, P.n);
    RBD_LAUNCH_CHECK();
    update_kernel<kInit><<<P.up_ncb, 256, 0, s>>>(P.n, st, 0, l2, up_groups, tickets, e2, base2, T, P.n, flist,
                                                  bres_v, bres_i, pivots, err_hist, start, tol, rel);
    RBD_LAUNCH_CHECK();
    prof_end(RBD_PHASE_INIT, s);

    // A = I: lagged reorthogonalisation, one pass over Y per step.  v1 and h2
    // alternate between two buffers by the parity of the step.
    double* const v1s[2] = {v1, v2};
    double* const h2s[2] = {h2, h2 + RBD_MAX_D + 1};
    // the basis is kept in Y itself, or in FP32 in the workspace (copied out by the epilogue)
    float* const Yf = P.y32 ? reinterpret_cast<float*>(ws + P.o_yf) : nullptr;
    auto identity_steps = [&](auto* Yb, int d0, int d1) -> int {
        using Tb = std::remove_pointer_t<decltype(Yb)>;
        const int64_t ldb = std::is_same<Tb, float>::value ? P.ldyf : P.d_max;
        for (int d = d0; d < d1; ++d) {
            const int c = d & 1;
            const int kc = kc_for(d);
            prof_begin(RBD_PHASE_CGS1, s);
            // the FP64-basis pass reads x_p from X itself; the FP32-basis pass takes it gathered
            if constexpr (std::is_same<Tb, float>::value) {
                launch_gather<Tx>(P, X, ldx, st, xp, s);
                RBD_LAUNCH_CHECK();
            }
            switch (kc) {
                case 1: launch_cgs1_lag<1>(P, X, ldx, xp, Yb, T, st, d, v1s[c ^ 1], h2s[c ^ 1], v1s[c], ys, part, s); break;
                case 2: launch_cgs1_lag<2>(P, X, ldx, xp, Yb, T, st, d, v1s[c ^ 1], h2s[c ^ 1], v1s[c], ys, part, s); break;
                case 4: launch_cgs1_lag<4>(P, X, ldx, xp, Yb, T, st, d, v1s[c ^ 1], h2s[c ^ 1], v1s[c], ys, part, s); break;
                case 8: launch_cgs1_lag<8>(P, X, ldx, xp, Yb, T, st, d, v1s[c ^ 1], h2s[c ^ 1], v1s[c], ys, part, s); break;
                default: launch_cgs1_lag<16>(P, X, ldx, xp, Yb, T, st, d, v1s[c ^ 1], h2s[c ^ 1], v1s[c], ys, part, s); break;
            }
            RBD_LAUNCH_CHECK();
            launch_sum_rows(st, part, std::max(P.D, 1), P.cg_S, P.cg_group, d + 1, l2, h2s[c], 0, s);
            RBD_LAUNCH_CHECK();
            prof_end(RBD_PHASE_CGS1, s);
            prof_begin(RBD_PHASE_CGS2, s);
            const int kp = d > 0 ? (int)cdiv(d, kTcorr) : 0;
            nu_tcorr_kernel<<<dim3(kp ? (unsigned)cdiv(P.n, 256) : 1u, (unsigned)std::max(kp, 1)), 256, 0, s>>>(
                st, h2s[c], d, T, P.n, P.n, part + (int64_t)P.sc_S * P.n);
            RBD_LAUNCH_CHECK();
            prof_end(RBD_PHASE_CGS2, s);
            prof_begin(RBD_PHASE_XSCAN, s);
            launch_xscan<Tx, kScanDot>(P, X, ldx, v1s[c], st, Y, -1, part, vec_ok, nt, s);
            RBD_LAUNCH_CHECK();
            prof_end(RBD_PHASE_XSCAN, s);
            prof_begin(RBD_PHASE_UPDATE, s);
            const int rows = P.sc_S + kp;
            const int groups = (int)cdiv(rows, up_per);
            reduce_rows_kernel<<<dim3((unsigned)cdiv(P.n, 256), (unsigned)groups), 256, 0, s>>>(st, part, P.n, rows,
                                                                                               up_per, P.n, l2, P.n);
            RBD_LAUNCH_CHECK();
            update_kernel<kStep><<<P.up_ncb, 256, 0, s>>>(P.n, st, d, l2, groups, tickets, e2, base2, T, P.n,
                                                          flist, bres_v, bres_i, pivots, err_hist, start, tol, rel);
            RBD_LAUNCH_CHECK();
            prof_end(RBD_PHASE_UPDATE, s);
            prof_begin(RBD_PHASE_RESID, s);
            // an exact refresh of this step needs Y(:, d): write it now (skipped when nothing is queued)
            launch_ycol_kc<false>(kc, P, Yb, st, d, v1s[0], v1s[1], h2s[0], h2s[1], ys, s);
            RBD_LAUNCH_CHECK();
            resid_mfma_kernel<Tx, false, Tb><<<P.rc_grid, 256, 0, s>>>(X, ldx, P.m, Yb, ldb, d + 1, T, P.n, flist, &st->nflag, 0,
                                                        P.rc_rows, P.rc_S, rpart, P.n, nullptr);
            RBD_LAUNCH_CHECK();
            prof_end(RBD_PHASE_RESID, s);
            prof_begin(RBD_PHASE_RESID_FINISH, s);
            resid_finish_kernel<<<P.rf_grid, 256, 0, s>>>(st, rpart, P.n, P.rc_S, flist, e2, base2, P.n, tickets, pivots,
                                                          err_hist, d);
            RBD_LAUNCH_CHECK();
            prof_end(RBD_PHASE_RESID_FINISH, s);
            prof_step(s);
        }
        return RBD_OK;
    };
    // With an FP32 basis the first kY32Switch steps still run on the FP64 basis in Y
    // (their passes are latency-bound: they gain nothing from fewer bytes), then the
    // complete columns are rounded into the FP32 basis and the rest run on it.
    const int dsw = Yf ? std::min(P.D, kY32Switch) : P.D;
    if (!W) {
        int rc = identity_steps(Y, 0, dsw);
        if (rc == RBD_OK && Yf && P.D > dsw) {
            static_assert(kY32Switch - 8 <= 128, "y32_switch_kernel copies at most 128 columns per row");
            y32_switch_kernel<<<(unsigned)cdiv(P.m, 2), 256, 0, s>>>(st, Y, P.d_max, Yf, P.ldyf, P.m, kY32Switch - 8);
            RBD_LAUNCH_CHECK();
            rc = identity_steps(Yf, dsw, P.D);
        }
        if (rc != RBD_OK) return rc;
    }
    // diagonal A: two passes over Y per step (M = Y'WY kept up to date)
    double* const avec = h2 + RBD_MAX_D + 1;     // a = Y'(w . v1) and sum w v1^2
    const int64_t ldp = std::max(P.D, 1);
    for (int d = 0; W && d < P.D; ++d) {
        const int kc = kc_for(d);
        prof_begin(RBD_PHASE_CGS1, s);
        launch_gather<Tx>(P, X, ldx, st, xp, s);
        RBD_LAUNCH_CHECK();
        switch (kc) {
            case 1: launch_cgs1w<1>(P, xp, Y, T, st, d, w, ys, v1, part, s); break;
            case 2: launch_cgs1w<2>(P, xp, Y, T, st, d, w, ys, v1, part, s); break;
            case 4: launch_cgs1w<4>(P, xp, Y, T, st, d, w, ys, v1, part, s); break;
            case 8: launch_cgs1w<8>(P, xp, Y, T, st, d, w, ys, v1, part, s); break;
            default: launch_cgs1w<16>(P, xp, Y, T, st, d, w, ys, v1, part, s); break;
        }
        RBD_LAUNCH_CHECK();
        launch_sum_rows(st, part, ldp, P.cg_S, P.cg_group, d + 1, l2, h2, 0, s);
        RBD_LAUNCH_CHECK();
        launch_sum_rows(st, part + (int64_t)P.cg_S * ldp, ldp, P.cg_S, P.cg_group, d + 1, l2, avec, 0, s);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_CGS1, s);
        prof_begin(RBD_PHASE_CGS2, s);
        if (d > 0) {
            mv_kernel<<<(unsigned)cdiv(d, 4), 256, 0, s>>>(st, Mw, ldp, d, h2, mh);
            RBD_LAUNCH_CHECK();
        }
        nuw_kernel<<<1, 256, 0, s>>>(st, h2, avec, mh, d, hw, Mw, ldp);
        RBD_LAUNCH_CHECK();
        switch (kc) {
            case 1: launch_gvec2<1>(P, Y, st, d, v1, h2, hw, w, ys, v2, g, s); break;
            case 2: launch_gvec2<2>(P, Y, st, d, v1, h2, hw, w, ys, v2, g, s); break;
            case 4: launch_gvec2<4>(P, Y, st, d, v1, h2, hw, w, ys, v2, g, s); break;
            case 8: launch_gvec2<8>(P, Y, st, d, v1, h2, hw, w, ys, v2, g, s); break;
            default: launch_gvec2<16>(P, Y, st, d, v1, h2, hw, w, ys, v2, g, s); break;
        }
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_CGS2, s);
        prof_begin(RBD_PHASE_XSCAN, s);
        launch_xscan<Tx, kScanDot2>(P, X, ldx, v2, st, Y, -1, part, vec_ok, nt, s, g);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_XSCAN, s);
        prof_begin(RBD_PHASE_UPDATE, s);
        reduce_rows_kernel<<<red_grid_step, 256, 0, s>>>(st, part, nw, P.sc_S, up_per, nw, l2, nw);
        RBD_LAUNCH_CHECK();
        update_kernel<kStepW><<<P.up_ncb, 256, 0, s>>>(P.n, st, d, l2, up_groups, tickets, e2, base2, T, P.n, flist,
                                                       bres_v, bres_i, pivots, err_hist, start, tol, rel);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_UPDATE, s);
        prof_begin(RBD_PHASE_RESID, s);
        // an exact refresh of this step needs Y(:, 0:d+1) in Y (skipped when nothing is queued)
        launch_ys_flush<false>(P, Y, st, d + 1, ys, s);
        RBD_LAUNCH_CHECK();
        resid_mfma_kernel<Tx><<<P.rc_grid, 256, 0, s>>>(X, ldx, P.m, Y, P.d_max, d + 1, T, P.n, flist, &st->nflag, 0,
                                                    P.rc_rows, P.rc_S, rpart, P.n, w);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_RESID, s);
        prof_begin(RBD_PHASE_RESID_FINISH, s);
        resid_finish_kernel<<<P.rf_grid, 256, 0, s>>>(st, rpart, P.n, P.rc_S, flist, e2, base2, P.n, tickets, pivots,
                                                      err_hist, d);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_RESID_FINISH, s);
        prof_step(s);
    }
    const int64_t work = std::max<int64_t>(P.m, P.n) + (int64_t)P.d_max;
    const int eg = (int)std::min<int64_t>(4096, cdiv(work, 256));
    prof_begin(RBD_PHASE_EPILOGUE, s);
    if (W) {
        launch_ys_flush<true>(P, Y, st, 0, ys, s);
        RBD_LAUNCH_CHECK();
    } else {
        // the last basis vector is still implicit: write it (into the FP64 basis when the
        // fit ended within its first dsw columns, else into the FP32 one)
        launch_ycol_kc<true>(kc_for(std::max(dsw - 1, 0)), P, Y, st, dsw, v1s[0], v1s[1], h2s[0], h2s[1], ys, s);
        RBD_LAUNCH_CHECK();
        if (Yf && P.D > dsw) {
            launch_ycol_kc<true>(kc_for(std::max(P.D - 1, 0)), P, Yf, st, dsw, v1s[0], v1s[1], h2s[0], h2s[1], ys,
                                 s);
            RBD_LAUNCH_CHECK();
        }
    }
    epilogue_kernel<<<eg, 256, 0, s>>>(st, e2, col_err, P.n, Y, P.m, P.d_max, T, pivots, err_hist, d_out, status,
                                       stop_reason, Yf, P.ldyf, dsw);
    RBD_LAUNCH_CHECK();
    prof_end(RBD_PHASE_EPILOGUE, s);
    return RBD_OK;
}

// ---------------------------------------------------------------------------
// General SPD A (section 3.2) in CSR form.  Same loop as the diagonal case,
// with A xi from a sparse product.  Exact refreshes need the residual columns
// themselves (r' A r), so they run in chunks of queued columns: every step
// enqueues the chunks for the longest possible queue, and each chunk reads the
// queue's length on the device and exits at once when it has nothing to do,
// so the host never waits on the stream.
// ---------------------------------------------------------------------------
struct SpdPlan {
    FitPlan F;
    int q_rows = 0, q_S = 0, cq = 0;
    size_t o_u, o_rbuf, o_qpart, total;
};

bool make_spd_plan(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, SpdPlan* P) {
    if (!make_fit_plan(m, n, d_max, xt, &P->F)) return false;
    P->q_rows = (int)std::max<int64_t>(64, cdiv(m, 2048));
    P->q_S = (int)cdiv(m, P->q_rows);
    // residual chunk: about 2 GB of FP64 columns, 64 .. 1024 of them
    int64_t c = ((int64_t)1 << 31) / (8 * m);
    c = std::max<int64_t>(64, std::min<int64_t>(1024, c / 64 * 64));
    c = std::min<int64_t>(c, cdiv(n, 64) * 64);
    P->cq = (int)c;
    size_t o = P->F.total;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    P->o_u = take(8 * (size_t)m);
    P->o_rbuf = take(8 * (size_t)m * P->cq);
    P->o_qpart = take(8 * (size_t)P->q_S * n);
    P->total = o;
    return true;
}

template <typename Tx>
int fit_spd_typed(const SpdPlan& Q, const Tx* X, int64_t ldx, Csr A, double tol, int rel, int64_t start, double* Y,
                  double* T, int64_t* pivots, double* col_err, double* err_hist, int32_t* d_out, int32_t* status,
                  int32_t* stop_reason, char* ws, hipStream_t s) {
    const FitPlan& P = Q.F;
    State* st = reinterpret_cast<State*>(ws + P.o_state);
    unsigned* tickets = reinterpret_cast<unsigned*>(ws + P.o_tickets);
    double* e2 = reinterpret_cast<double*>(ws + P.o_e2);
    double* base2 = reinterpret_cast<double*>(ws + P.o_base2);
    int* flist = reinterpret_cast<int*>(ws + P.o_flist);
    double* bres_v = reinterpret_cast<double*>(ws + P.o_bres_v);
    int64_t* bres_i = reinterpret_cast<int64_t*>(ws + P.o_bres_i);
    double* v1 = reinterpret_cast<double*>(ws + P.o_v1);
    double* v2 = reinterpret_cast<double*>(ws + P.o_v2);
    double* h2 = reinterpret_cast<double*>(ws + P.o_h2);
    double* part = reinterpret_cast<double*>(ws + P.o_part);
    double* l2 = reinterpret_cast<double*>(ws + P.o_l2);
    double* g = reinterpret_cast<double*>(ws + P.o_g);
    double* hw = reinterpret_cast<double*>(ws + P.o_hw);
    double* xp = reinterpret_cast<double*>(ws + P.o_xp);
    double* u = reinterpret_cast<double*>(ws + Q.o_u);
    double* Ma = reinterpret_cast<double*>(ws + P.o_M);      // M = Y'AY
    double* mh = reinterpret_cast<double*>(ws + P.o_mh);
    double* const yu = h2 + RBD_MAX_D + 1;                     // Y'(A v1) and v1'A v1
    double* ys = reinterpret_cast<double*>(ws + P.o_ys);
    double* rbuf = reinterpret_cast<double*>(ws + Q.o_rbuf);
    double* qpart = reinterpret_cast<double*>(ws + Q.o_qpart);
    const int64_t nw = 2 * P.n;
    const int N = Ld<Tx>::N;
    const int vec_ok = (ldx % N == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    const bool nt = (double)P.m * (double)ldx * sizeof(Tx) > 512.0 * 1024 * 1024;

    prof_fit_begin(s);
    init_state_kernel<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(P.ntickets, 256))), 256, 0, s>>>(
        st, tickets, P.ntickets, P.D);
    RBD_LAUNCH_CHECK();
    // pre-computation of diag(X'AX) (section 3.3)
    prof_begin(RBD_PHASE_COLNORM, s);
    csr_xax_kernel<Tx><<<dim3((unsigned)cdiv(P.n, 256), (unsigned)P.sc_S), 256, 0, s>>>(X, ldx, P.m, P.n, A, P.sc_rows,
                                                                                       part, st);
    RBD_LAUNCH_CHECK();
    prof_end(RBD_PHASE_COLNORM, s);
    prof_begin(RBD_PHASE_INIT, s);
    const int up_per = (int)cdiv(P.sc_S, P.up_SG);
    const int up_groups = (int)cdiv(P.sc_S, up_per);
    reduce_rows_kernel<<<dim3((unsigned)cdiv(P.n, 256), (unsigned)up_groups), 256, 0, s>>>(nullptr, part, P.n, P.sc_S,
                                                                                          up_per, P.n, l2, P.n);
    RBD_LAUNCH_CHECK();
    update_kernel<kInit><<<P.up_ncb, 256, 0, s>>>(P.n, st, 0, l2, up_groups, tickets, e2, base2, T, P.n, flist,
                                                  bres_v, bres_i, pivots, err_hist, start, tol, rel);
    RBD_LAUNCH_CHECK();
    prof_end(RBD_PHASE_INIT, s);

    const int64_t ldp = std::max(P.D, 1);
    const unsigned sp_grid = (unsigned)std::min<int64_t>(16384, cdiv(P.m, 256));
    for (int d = 0; d < P.D; ++d) {
        const int kc = kc_for(d);
        prof_begin(RBD_PHASE_CGS1, s);
        launch_gather<Tx>(P, X, ldx, st, xp, s);
        switch (kc) {
            case 1: launch_cgs1<1>(P, xp, Y, T, st, d, ys, v1, part, s); break;
            case 2: launch_cgs1<2>(P, xp, Y, T, st, d, ys, v1, part, s); break;
            case 4: launch_cgs1<4>(P, xp, Y, T, st, d, ys, v1, part, s); break;
            case 8: launch_cgs1<8>(P, xp, Y, T, st, d, ys, v1, part, s); break;
            default: launch_cgs1<16>(P, xp, Y, T, st, d, ys, v1, part, s); break;
        }
        RBD_LAUNCH_CHECK();
        launch_sum_rows(st, part, ldp, P.cg_S, P.cg_group, d + 1, l2, h2, 0, s);
        RBD_LAUNCH_CHECK();
        nu_lag_kernel<<<1, 256, 0, s>>>(st, h2, d);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_CGS1, s);
        prof_begin(RBD_PHASE_CGS2, s);
        // u = A v1; second pass: xi, v2 and Y'u, v1'u; then hw, ||xi||_A^2, M
        spmv_kernel<false><<<sp_grid, 256, 0, s>>>(st, A, P.m, v1, u);
        RBD_LAUNCH_CHECK();
        switch (kc) {
            case 1: launch_cgs2u<1>(P, Y, st, d, v1, h2, u, ys, v2, part, s); break;
            case 2: launch_cgs2u<2>(P, Y, st, d, v1, h2, u, ys, v2, part, s); break;
            case 4: launch_cgs2u<4>(P, Y, st, d, v1, h2, u, ys, v2, part, s); break;
            case 8: launch_cgs2u<8>(P, Y, st, d, v1, h2, u, ys, v2, part, s); break;
            default: launch_cgs2u<16>(P, Y, st, d, v1, h2, u, ys, v2, part, s); break;
        }
        RBD_LAUNCH_CHECK();
        launch_sum_rows(st, part, ldp, P.cg_S, P.cg_group, d + 1, l2, yu, 0, s);
        RBD_LAUNCH_CHECK();
        if (d > 0) {
            mv_kernel<<<(unsigned)cdiv(d, 4), 256, 0, s>>>(st, Ma, ldp, d, h2, mh);
            RBD_LAUNCH_CHECK();
        }
        nuw_kernel<<<1, 256, 0, s>>>(st, h2, yu, mh, d, hw, Ma, ldp);
        RBD_LAUNCH_CHECK();
        spmv_kernel<true><<<sp_grid, 256, 0, s>>>(st, A, P.m, v2, g);
        RBD_LAUNCH_CHECK();
        const int kp = d > 0 ? (int)cdiv(d, kTcorr) : 0;
        if (kp) {
            tcorr2_kernel<<<dim3((unsigned)cdiv(P.n, 256), (unsigned)kp), 256, 0, s>>>(
                st, hw, d, T, P.n, P.n, part + (int64_t)P.sc_S * nw);
            RBD_LAUNCH_CHECK();
        }
        prof_end(RBD_PHASE_CGS2, s);
        prof_begin(RBD_PHASE_XSCAN, s);
        launch_xscan<Tx, kScanDot2>(P, X, ldx, v2, st, Y, -1, part, vec_ok, nt, s, g);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_XSCAN, s);
        prof_begin(RBD_PHASE_UPDATE, s);
        const int rows = P.sc_S + kp;
        const int groups = (int)cdiv(rows, up_per);
        reduce_rows_kernel<<<dim3((unsigned)cdiv(nw, 256), (unsigned)groups), 256, 0, s>>>(st, part, nw, rows, up_per,
                                                                                          nw, l2, nw);
        RBD_LAUNCH_CHECK();
        update_kernel<kStepW><<<P.up_ncb, 256, 0, s>>>(P.n, st, d, l2, groups, tickets, e2, base2, T, P.n, flist,
                                                       bres_v, bres_i, pivots, err_hist, start, tol, rel);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_UPDATE, s);
        // exact refreshes: chunks for every possible queue length, each sized on
        // the device from the queue's length (an empty chunk, or a step with
        // nothing queued, or a step after the loop has stopped, costs one empty
        // launch per kernel), so the host never waits
        prof_begin(RBD_PHASE_RESID, s);
        launch_ys_flush<false>(P, Y, st, d + 1, ys, s);
        RBD_LAUNCH_CHECK();
        for (int c0 = 0; c0 < P.n; c0 += Q.cq) {
            const int cc = (int)std::min<int64_t>(Q.cq, P.n - c0);      // at most this many queued columns
            const unsigned grid = (unsigned)std::min<int64_t>(2048, cdiv(cc, 64) * P.rc_S);
            resid_mfma_kernel<Tx, true><<<grid, 256, 0, s>>>(X, ldx, P.m, Y, P.d_max, d + 1, T, P.n, flist + c0,
                                                              &st->nflag, 0, P.rc_rows, P.rc_S, nullptr, 0, nullptr,
                                                              rbuf, Q.cq, c0, Q.cq);
            RBD_LAUNCH_CHECK();
            csr_quad_kernel<<<dim3((unsigned)cdiv(cc, 64), (unsigned)Q.q_S), 64 * kQuadGroups, 0, s>>>(
                rbuf, Q.cq, P.m, &st->nflag, Q.cq, A, Q.q_rows, qpart, P.n, c0);
            RBD_LAUNCH_CHECK();
        }
        prof_end(RBD_PHASE_RESID, s);
        prof_begin(RBD_PHASE_RESID_FINISH, s);
        resid_finish_kernel<<<P.rf_grid, 256, 0, s>>>(st, qpart, P.n, Q.q_S, flist, e2, base2, P.n, tickets,
                                                      pivots, err_hist, d);
        RBD_LAUNCH_CHECK();
        prof_end(RBD_PHASE_RESID_FINISH, s);
        prof_step(s);
    }
    const int64_t work = std::max<int64_t>(P.m, P.n) + (int64_t)P.d_max;
    const int eg = (int)std::min<int64_t>(4096, cdiv(work, 256));
    prof_begin(RBD_PHASE_EPILOGUE, s);
    launch_ys_flush<true>(P, Y, st, 0, ys, s);
    RBD_LAUNCH_CHECK();
    epilogue_kernel<<<eg, 256, 0, s>>>(st, e2, col_err, P.n, Y, P.m, P.d_max, T, pivots, err_hist, d_out, status,
                                       stop_reason);
    RBD_LAUNCH_CHECK();
    prof_end(RBD_PHASE_EPILOGUE, s);
    return RBD_OK;
}

// ---------------------------------------------------------------------------
struct ProjPlan {
    size_t part_elems = 0;      // split-k partials of C = Y'V
    int rc_rows = 0, rc_S = 0, rc_grid = 0;
    int rs_per = 0, rs_groups = 0;  // residual partials summed in groups of rs_per slabs, then the groups
    size_t o_part, o_rpart, o_rgroup, total;
};

bool make_proj_plan(int64_t m, int32_t d, int64_t k, ProjPlan* P) {
    if (m < 1 || d < 1 || k < 1 || d > RBD_MAX_D || k >= (int64_t)INT32_MAX) return false;
    // room for the k-splits that bring the product to about 1024 workgroups
    P->part_elems = (size_t)std::min<int64_t>((int64_t)kPartElems, std::min<int64_t>(1024, cdiv(m, 1024)) * d * k);
    // residual norms: row slabs of a multiple of 128 rows, enough for about 4096 (tile, slab) items
    const int64_t slabs = std::max<int64_t>(32, cdiv(4096, cdiv(k, 64)));
    int64_t rrow = std::min<int64_t>(std::max<int64_t>(128, cdiv(cdiv(m, slabs), 128) * 128), INT32_MAX / 2);
    P->rc_rows = (int)rrow;
    P->rc_S = (int)cdiv(m, rrow);
    P->rc_grid = (int)std::min<int64_t>(2048, cdiv(k, 64) * P->rc_S);
    P->rs_per = std::min(P->rc_S, 64);
    P->rs_groups = (int)cdiv(P->rc_S, P->rs_per);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    P->o_part = take(8 * P->part_elems);
    P->o_rpart = take(8 * (size_t)P->rc_S * k);
    P->o_rgroup = take(8 * (size_t)P->rs_groups * k);
    P->total = o;
    return true;
}

template <typename Tv>
int project_typed(const ProjPlan& P, const double* Y, int64_t ldy, int64_t m, int d, const Tv* V, int64_t k,
                  int64_t ldv, double* Tv_out, double* err_v, char* ws, hipStream_t s) {
    double* part = reinterpret_cast<double*>(ws + P.o_part);
    double* rpart = reinterpret_cast<double*>(ws + P.o_rpart);
    double* rgroup = reinterpret_cast<double*>(ws + P.o_rgroup);
    // coefficients on the FP64 matrix cores (split-k partials summed in a fixed order)
    if (proj_mfma<Tv>(Y, ldy, m, d, V, ldv, k, Tv_out, k, part, P.part_elems, s) != hipSuccess) return RBD_EDEVICE;
    resid_mfma_kernel<Tv><<<P.rc_grid, 256, 0, s>>>(V, ldv, m, Y, ldy, d, Tv_out, k, nullptr, nullptr, (int)k, P.rc_rows,
                                               P.rc_S, rpart, k, nullptr);
    RBD_LAUNCH_CHECK();
    // slab partials -> group sums -> norms, every sum in ascending order (two levels keep
    // each thread's serial chain short when k is small and the slabs are many)
    const double* rsum = rpart;
    if (P.rs_groups > 1) {
        reduce_rows_kernel<<<dim3((unsigned)cdiv(k, 256), (unsigned)P.rs_groups), 256, 0, s>>>(
            nullptr, rpart, k, P.rc_S, P.rs_per, k, rgroup, k);
        RBD_LAUNCH_CHECK();
        rsum = rgroup;
    }
    sum_rows_kernel<<<(unsigned)std::min<int64_t>(4096, cdiv(k, 256)), 256, 0, s>>>(rsum, P.rs_groups > 1 ? P.rs_groups : P.rc_S,
                                                                                     k, err_v, 1);
    RBD_LAUNCH_CHECK();
    return RBD_OK;
}

}  // namespace

// Workspace of rbd_fit_noalloc: a fixed device array in this code object, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it only stands for the symbol): its
// device address is looked up once per device with that device current, and
// only that address is used.
static __device__ __align__(256) unsigned char scratch[RBD_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return RBD_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr ||
            reinterpret_cast<uintptr_t>(ptr) % kAlign != 0) {
            (void)hipGetLastError();
            return RBD_EDEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RBD_OK;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int rbd_fit_workspace_size(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, size_t* bytes) {
    if (!bytes) return RBD_EINVAL;
    FitPlan P;
    if (!make_fit_plan(m, n, d_max, xt, &P)) return RBD_EINVAL;
    *bytes = P.total;
    return RBD_OK;
}

// Host-side argument checks shared by rbd_fit and rbd_fit_noalloc (no device call).
static int check_fit_args(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, double tol,
                          rbd_tol_mode mode, int32_t d_max, int64_t start, const double* Y, const double* T,
                          const int64_t* pivots, const double* col_err, const double* err_hist, const int32_t* d_out,
                          const int32_t* status, FitPlan* P, int basis = RBD_BASIS_F64) {
    if (!make_fit_plan(m, n, d_max, xt, P, basis)) return RBD_EINVAL;
    if (!X || !Y || !T || !pivots || !col_err || !err_hist || !d_out || !status) return RBD_EINVAL;
    if (ldx < n) return RBD_EINVAL;
    if (!(tol >= 0.0) || tol == HUGE_VAL) return RBD_EINVAL;
    if (mode != RBD_TOL_ABS && mode != RBD_TOL_REL) return RBD_EINVAL;
    if (start >= n) return RBD_EINVAL;
    return RBD_OK;
}

static int fit_entry(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, double tol, rbd_tol_mode mode,
                     int32_t d_max, int64_t start, double* Y, double* T, int64_t* pivots, double* col_err,
                     double* err_hist, int32_t* d_out, int32_t* status, int32_t* stop_reason, void* workspace,
                     size_t workspace_bytes, void* stream, const double* w, int basis = RBD_BASIS_F64) {
    FitPlan P;
    const int rc = check_fit_args(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist,
                                  d_out, status, &P, basis);
    if (rc != RBD_OK) return rc;
    if (w && P.y32) return RBD_EINVAL;          // the FP32 basis is for A = I only
    if (!workspace) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return RBD_EINVAL;
    if (workspace_bytes < P.total) return RBD_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    const int rel = (mode == RBD_TOL_REL);
    switch (xt) {
        case RBD_F32:
            return fit_typed<float>(P, static_cast<const float*>(X), ldx, tol, rel, start, Y, T, pivots, col_err,
                                    err_hist, d_out, status, stop_reason, ws, s, w);
        case RBD_F64:
            return fit_typed<double>(P, static_cast<const double*>(X), ldx, tol, rel, start, Y, T, pivots, col_err,
                                     err_hist, d_out, status, stop_reason, ws, s, w);
        case RBD_BF16:
            return fit_typed<bf16_t>(P, static_cast<const bf16_t*>(X), ldx, tol, rel, start, Y, T, pivots, col_err,
                                     err_hist, d_out, status, stop_reason, ws, s, w);
        case RBD_F16:
            return fit_typed<f16_t>(P, static_cast<const f16_t*>(X), ldx, tol, rel, start, Y, T, pivots, col_err,
                                    err_hist, d_out, status, stop_reason, ws, s, w);
    }
    return RBD_EINVAL;
}

int rbd_fit(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, double tol, rbd_tol_mode mode,
            int32_t d_max, int64_t start, double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
            int32_t* d_out, int32_t* status, int32_t* stop_reason, void* workspace, size_t workspace_bytes,
            void* stream) {
    return fit_entry(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist, d_out, status,
                     stop_reason, workspace, workspace_bytes, stream, nullptr);
}

int rbd_fit_basis_workspace_size(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, rbd_basis basis,
                                 size_t* bytes) {
    if (!bytes) return RBD_EINVAL;
    FitPlan P;
    if (!make_fit_plan(m, n, d_max, xt, &P, (int)basis)) return RBD_EINVAL;
    *bytes = P.total;
    return RBD_OK;
}

int rbd_fit_basis(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, double tol, rbd_tol_mode mode,
                  int32_t d_max, int64_t start, rbd_basis basis, double* Y, double* T, int64_t* pivots,
                  double* col_err, double* err_hist, int32_t* d_out, int32_t* status, int32_t* stop_reason,
                  void* workspace, size_t workspace_bytes, void* stream) {
    return fit_entry(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist, d_out, status,
                     stop_reason, workspace, workspace_bytes, stream, nullptr, (int)basis);
}

int rbd_fit_noalloc(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, double tol,
                    rbd_tol_mode mode, int32_t d_max, int64_t start, double* Y, double* T, int64_t* pivots,
                    double* col_err, double* err_hist, int32_t* d_out, int32_t* status, int32_t* stop_reason,
                    void* stream) {
    FitPlan P;
    const int rc = check_fit_args(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist,
                                  d_out, status, &P);
    if (rc != RBD_OK) return rc;
    if (P.total > RBD_NOALLOC_MAX_BYTES) return RBD_ETOOLARGE;
    void* ws = nullptr;
    const int rs = noalloc_scratch(&ws);
    if (rs != RBD_OK) return rs;
    return fit_entry(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist, d_out, status,
                     stop_reason, ws, RBD_NOALLOC_MAX_BYTES, stream, nullptr);
}

int rbd_fit_weighted(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, const double* weights,
                     double tol, rbd_tol_mode mode, int32_t d_max, int64_t start, double* Y, double* T,
                     int64_t* pivots, double* col_err, double* err_hist, int32_t* d_out, int32_t* status,
                     int32_t* stop_reason, void* workspace, size_t workspace_bytes, void* stream) {
    if (!weights) return RBD_EINVAL;
    return fit_entry(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist, d_out, status,
                     stop_reason, workspace, workspace_bytes, stream, weights);
}

struct rbd_fit_graph_s {
    hipGraphExec_t exec;
};

int rbd_fit_graph_create(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, const double* weights,
                         double tol, rbd_tol_mode mode, int32_t d_max, int64_t start, double* Y, double* T,
                         int64_t* pivots, double* col_err, double* err_hist, int32_t* d_out, int32_t* status,
                         int32_t* stop_reason, void* workspace, size_t workspace_bytes, void* stream,
                         rbd_fit_graph* out) {
    if (!out || !stream) return RBD_EINVAL;
    *out = nullptr;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return RBD_EDEVICE;
    const int rc = fit_entry(X, xt, m, n, ldx, tol, mode, d_max, start, Y, T, pivots, col_err, err_hist, d_out,
                             status, stop_reason, workspace, workspace_bytes, stream, weights);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc != RBD_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rc != RBD_OK ? rc : RBD_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess || !exec) return RBD_EDEVICE;
    rbd_fit_graph g = new (std::nothrow) rbd_fit_graph_s{exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return RBD_EDEVICE;
    }
    *out = g;
    return RBD_OK;
}

int rbd_fit_graph_launch(rbd_fit_graph graph, void* stream) {
    if (!graph) return RBD_EINVAL;
    return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? RBD_OK : RBD_EDEVICE;
}

int rbd_fit_graph_destroy(rbd_fit_graph graph) {
    if (!graph) return RBD_OK;
    const hipError_t e = hipGraphExecDestroy(graph->exec);
    delete graph;
    return e == hipSuccess ? RBD_OK : RBD_EDEVICE;
}

int rbd_fit_spd_workspace_size(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, size_t* bytes) {
    if (!bytes) return RBD_EINVAL;
    SpdPlan Q;
    if (!make_spd_plan(m, n, d_max, xt, &Q)) return RBD_EINVAL;
    *bytes = Q.total;
    return RBD_OK;
}

int rbd_fit_spd(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, const int64_t* a_indptr,
                const int32_t* a_indices, const double* a_values, int64_t a_nnz, double tol, rbd_tol_mode mode,
                int32_t d_max, int64_t start, double* Y, double* T, int64_t* pivots, double* col_err,
                double* err_hist, int32_t* d_out, int32_t* status, int32_t* stop_reason, void* workspace,
                size_t workspace_bytes, void* stream) {
    SpdPlan Q;
    if (!make_spd_plan(m, n, d_max, xt, &Q)) return RBD_EINVAL;
    if (m >= (int64_t)INT32_MAX) return RBD_EINVAL;
    if (!X || !Y || !T || !pivots || !col_err || !err_hist || !d_out || !status || !workspace) return RBD_EINVAL;
    if (!a_indptr || (a_nnz > 0 && (!a_indices || !a_values)) || a_nnz < 0) return RBD_EINVAL;
    if (ldx < n) return RBD_EINVAL;
    if (!(tol >= 0.0) || tol == HUGE_VAL) return RBD_EINVAL;
    if (mode != RBD_TOL_ABS && mode != RBD_TOL_REL) return RBD_EINVAL;
    if (start >= n) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return RBD_EINVAL;
    if (workspace_bytes < Q.total) return RBD_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    const int rel = (mode == RBD_TOL_REL);
    const Csr A{a_indptr, a_indices, a_values, a_nnz};
    switch (xt) {
        case RBD_F32:
            return fit_spd_typed<float>(Q, static_cast<const float*>(X), ldx, A, tol, rel, start, Y, T, pivots,
                                        col_err, err_hist, d_out, status, stop_reason, ws, s);
        case RBD_F64:
            return fit_spd_typed<double>(Q, static_cast<const double*>(X), ldx, A, tol, rel, start, Y, T, pivots,
                                         col_err, err_hist, d_out, status, stop_reason, ws, s);
        case RBD_BF16:
            return fit_spd_typed<bf16_t>(Q, static_cast<const bf16_t*>(X), ldx, A, tol, rel, start, Y, T, pivots,
                                         col_err, err_hist, d_out, status, stop_reason, ws, s);
        case RBD_F16:
            return fit_spd_typed<f16_t>(Q, static_cast<const f16_t*>(X), ldx, A, tol, rel, start, Y, T, pivots,
                                        col_err, err_hist, d_out, status, stop_reason, ws, s);
    }
    return RBD_EINVAL;
}

int rbd_project_workspace_size(int64_t m, int32_t d, int64_t k, rbd_dtype vt, size_t* bytes) {
    if (!bytes || elem_bytes(vt) == 0) return RBD_EINVAL;
    ProjPlan P;
    if (!make_proj_plan(m, d, k, &P)) return RBD_EINVAL;
    *bytes = P.total;
    return RBD_OK;
}

int rbd_project(const double* Y, int64_t ldy, int64_t m, int32_t d, const void* V, rbd_dtype vt, int64_t k,
                int64_t ldv, double* Tv, double* err_v, void* workspace, size_t workspace_bytes, void* stream) {
    ProjPlan P;
    if (elem_bytes(vt) == 0 || !make_proj_plan(m, d, k, &P)) return RBD_EINVAL;
    if (!Y || !V || !Tv || !err_v || !workspace) return RBD_EINVAL;
    if (ldy < d || ldv < k) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return RBD_EINVAL;
    if (workspace_bytes < P.total) return RBD_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    switch (vt) {
        case RBD_F32:
            return project_typed<float>(P, Y, ldy, m, d, static_cast<const float*>(V), k, ldv, Tv, err_v, ws, s);
        case RBD_F64:
            return project_typed<double>(P, Y, ldy, m, d, static_cast<const double*>(V), k, ldv, Tv, err_v, ws, s);
        case RBD_BF16:
            return project_typed<bf16_t>(P, Y, ldy, m, d, static_cast<const bf16_t*>(V), k, ldv, Tv, err_v, ws, s);
        case RBD_F16:
            return project_typed<f16_t>(P, Y, ldy, m, d, static_cast<const f16_t*>(V), k, ldv, Tv, err_v, ws, s);
    }
    return RBD_EINVAL;
}

int rbd_profiler_begin(uint32_t phase_mask) {
    if (g_prof.on) return RBD_EINVAL;
    g_prof.on = true;
    g_prof.mask = phase_mask;
    g_prof.used = 0;
    g_prof.marks.clear();
    g_prof.steps.clear();
    g_prof.failed = false;
    return RBD_OK;
}

int rbd_profiler_end(double* phase_ms, int64_t* phase_launches, int32_t nphase, double* step_end_ms, int64_t nstep,
                     int64_t* nstep_out) {
    if (!g_prof.on) return RBD_EINVAL;
    g_prof.on = false;
    if (g_prof.failed) return RBD_EDEVICE;
    if (g_prof.used > 0 && hipEventSynchronize(g_prof.pool[g_prof.used - 1]) != hipSuccess) return RBD_EDEVICE;
    if (phase_ms)
        for (int i = 0; i < nphase; ++i) phase_ms[i] = 0.0;
    if (phase_launches)
        for (int i = 0; i < nphase; ++i) phase_launches[i] = 0;
    for (const auto& mk : g_prof.marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_prof.pool[mk.a], g_prof.pool[mk.b]) != hipSuccess) return RBD_EDEVICE;
        if (mk.phase < nphase) {
            if (phase_ms) phase_ms[mk.phase] += ms;
            if (phase_launches) phase_launches[mk.phase] += 1;
        }
    }
    const int64_t ns = (int64_t)g_prof.steps.size();
    if (nstep_out) *nstep_out = ns;
    if (step_end_ms) {
        for (int64_t i = 0; i < ns && i < nstep; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, g_prof.pool[g_prof.fit_start], g_prof.pool[g_prof.steps[i]]) != hipSuccess)
                return RBD_EDEVICE;
            step_end_ms[i] = ms;
        }
    }
    g_prof.used = 0;
    g_prof.marks.clear();
    g_prof.steps.clear();
    return RBD_OK;
}

int rbd_read_stream(const void* data, size_t bytes, int nontemporal, void* sink, void* stream) {
    if (!data || !sink || bytes == 0 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(data) % 16 != 0)
        return RBD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t nvec = (int64_t)(bytes / 16);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(nvec, 256)));
    const u32x4* v = reinterpret_cast<const u32x4*>(data);
    unsigned* out = reinterpret_cast<unsigned*>(sink);
    if (nontemporal) read_stream_kernel<true><<<grid, 256, 0, s>>>(v, nvec, 0x9e3779b9u, out);
    else read_stream_kernel<false><<<grid, 256, 0, s>>>(v, nvec, 0x9e3779b9u, out);
    RBD_LAUNCH_CHECK();
    return RBD_OK;
}

const char* rbd_status_string(int code) {
    switch (code) {
        case RBD_OK: return "ok";
        case RBD_EINVAL: return "invalid argument";
        case RBD_ENONFINITE: return "input holds a non-finite value";
        case RBD_EWORKSPACE: return "workspace too small";
        case RBD_EDEVICE: return "HIP launch or runtime error";
        case RBD_EMATRIX: return "sparse A holds an index outside its rows";
        case RBD_ETOOLARGE: return "the fit needs more workspace than rbd_fit_noalloc's fixed scratch";
    }
    return "unknown status";
}

const char* rbd_version(void) { return "rbd-gfx950 0.1"; }

}  // extern "C"
