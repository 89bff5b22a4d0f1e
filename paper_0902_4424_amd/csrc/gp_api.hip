// C ABI of the GPSS solver: handle, workspace, argument checks, launch
// sequence.  The iteration runs entirely on the device; the host enqueues
// `chunk` iterations at a time and reads one status word between chunks.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>

#include "gp_l1.h"
#include "gp_kernels.hpp"
#include "gp_wide.hpp"
#include "gp_internal.hpp"
#include "gp_verify.hpp"

using namespace gpl1;

// Fixed workspace of gp_l1_solve_noalloc: one copy per device, held until the
// process ends.  Host code never uses this name as an address; it works with
// the per-device address that gp_create looks up (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[GP_NOALLOC_SCRATCH_BYTES];

namespace gpl1 {

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `device`, looked up once.
static int setup_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return GP_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return GP_OK_TOL;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) { (void)hipGetLastError(); return GP_E_HIP; }
    g_scratch_ptr[device] = ptr;
    return GP_OK_TOL;
}

static void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

const char* status_name(int s) {
    switch (s) {
        case GP_OK_TOL: return "ok_tol";
        case GP_STATIONARY: return "stationary";
        case GP_MAX_ITER: return "max_iter";
        case GP_REACHED_TARGET: return "reached_target";
        case GP_BACKTRACK_LIMIT: return "backtrack_limit";
        case GP_E_ARG: return "bad argument";
        case GP_E_NONFINITE: return "non-finite value";
        case GP_E_HIP: return "HIP error";
        case GP_E_NOMEM: return "out of memory";
        case GP_E_UNSUPPORTED: return "unsupported shape";
    }
    return "unknown";
}

int fail(gp_handle h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(gp_handle h, hipError_t e, const char* where) {
    return fail(h, GP_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

int ensure_workspace(gp_handle h, size_t bytes) {
    if (bytes <= h->ws_bytes) return GP_OK_TOL;
    if (h->ws) {
        hipError_t e = hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
        if (e != hipSuccess) return hip_fail(h, e, "hipFree(workspace)");
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&h->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->ws = nullptr;
        return fail(h, GP_E_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    h->ws_bytes = want;
    return GP_OK_TOL;
}

int ensure_pinned(gp_handle h, size_t bytes) {
    if (bytes <= h->pin_bytes) return GP_OK_TOL;
    if (h->pin) {
        hipError_t e = hipHostFree(h->pin);
        h->pin = nullptr;
        h->pin_bytes = 0;
        if (e != hipSuccess) return hip_fail(h, e, "hipHostFree(pinned buffer)");
    }
    const size_t want = std::max(bytes, (size_t)1 << 16);
    hipError_t e = hipHostMalloc(&h->pin, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->pin = nullptr;
        return fail(h, GP_E_NOMEM, "pinned host allocation of " + std::to_string(want) + " bytes failed");
    }
    h->pin_bytes = want;
    return GP_OK_TOL;
}

int graph_stream(gp_handle h, hipStream_t user, hipStream_t* out) {
    *out = user;
    if (user) return GP_OK_TOL;
    // a graph cannot be captured on the null stream: run on the handle's own
    // stream, ordered after the caller's work
    hipError_t e;
    if (!h->gstream && (e = hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(h, e, "graph stream");
    if (!h->gevent && (e = hipEventCreateWithFlags(&h->gevent, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(h, e, "graph event");
    e = hipEventRecord(h->gevent, user);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->gstream, h->gevent, 0);
    if (e != hipSuccess) return hip_fail(h, e, "graph stream order");
    *out = h->gstream;
    return GP_OK_TOL;
}

int capture_graph(gp_handle h, hipStream_t s, hipGraphExec_t* exec, const std::function<void()>& enqueue) {
    if (*exec) { (void)hipGraphExecDestroy(*exec); *exec = nullptr; }
    hipGraph_t gr = nullptr;
    hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (ce != hipSuccess) return hip_fail(h, ce, "graph capture");
    enqueue();
    ce = hipStreamEndCapture(s, &gr);
    if (ce == hipSuccess) ce = hipGraphInstantiate(exec, gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    if (ce != hipSuccess) { *exec = nullptr; return hip_fail(h, ce, "graph instantiate"); }
    return GP_OK_TOL;
}

hipEvent_t prof_event(gp_handle h) {
    if (h->ev_used == (int)h->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->events.push_back(e);
    }
    return h->events[h->ev_used++];
}

// Sum the first `live` event pairs (launches enqueued after the solve stopped
// exit at once and are not counted).
double prof_collect(gp_handle h, int live, int* pairs) {
    double ms = 0.0;
    int np = 0;
    for (int i = 0; i + 1 < h->ev_used && np < live; i += 2) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->events[i], h->events[i + 1]) == hipSuccess) { ms += t; ++np; }
    }
    h->ev_used = 0;
    if (pairs) *pairs = np;
    return ms;
}

GPParams make_params(const gp_opts& o, double rho, double tol) {
    GPParams P;
    P.theta = o.theta;
    P.beta = o.beta;
    P.amin = o.alpha_min;
    P.amax = o.alpha_max;
    P.tau1 = o.tau1;
    P.f_target = o.f_target;
    P.tol = tol;
    P.rho = rho;
    P.M = o.M;
    P.Malpha = o.M_alpha;
    P.max_iter = o.max_iter;
    P.bt_cap = o.backtrack_cap;
    P.x0_fallback = o.x0_fallback ? 1 : 0;
    P.progress = nullptr;
    P.trace = nullptr;
    P.trace_cap = 0;
    return P;
}

int check_opts(gp_handle h, const gp_opts& o) {
    if (!(o.M >= 1 && o.M <= MAX_M)) return fail(h, GP_E_ARG, "opts.M must be in 1..16");
    if (!(o.theta > 0.0 && o.theta < 1.0)) return fail(h, GP_E_ARG, "opts.theta must be in (0,1)");
    if (!(o.beta > 0.0 && o.beta < 1.0)) return fail(h, GP_E_ARG, "opts.beta must be in (0,1)");
    if (!(o.alpha_min > 0.0 && o.alpha_min < o.alpha_max && std::isfinite(o.alpha_max)))
        return fail(h, GP_E_ARG, "need 0 < alpha_min < alpha_max < inf");
    if (!(o.tau1 > 0.0 && o.tau1 < 1.0)) return fail(h, GP_E_ARG, "opts.tau1 must be in (0,1)");
    if (o.trace && o.trace_cap <= 0) return fail(h, GP_E_ARG, "opts.trace needs opts.trace_cap > 0");
    if (!(o.M_alpha >= 0 && o.M_alpha <= MAX_RING - 1)) return fail(h, GP_E_ARG, "opts.M_alpha must be in 0..3");
    if (o.max_iter < 0) return fail(h, GP_E_ARG, "opts.max_iter must be >= 0");
    if (o.refresh_every < 0) return fail(h, GP_E_ARG, "opts.refresh_every must be >= 0");
    if (o.backtrack_cap < 0 || o.backtrack_cap > 1000) return fail(h, GP_E_ARG, "opts.backtrack_cap must be in 0..1000");
    if (o.chunk < 1) return fail(h, GP_E_ARG, "opts.chunk must be >= 1");
    if (std::isnan(o.f_target)) return fail(h, GP_E_ARG, "opts.f_target is NaN");
    if (o.profile < 0) return fail(h, GP_E_ARG, "opts.profile must be >= 0");
    if (o.graph && o.profile) return fail(h, GP_E_ARG, "opts.graph and opts.profile exclude each other");
    if (o.batch_splitk < 0 || o.batch_splitk % 32 != 0)
        return fail(h, GP_E_ARG, "opts.batch_splitk must be 0 or a positive multiple of 32");
    for (int t : {o.batch_rows_t, o.batch_cols_t})
        if (t != 0 && t != 256 && t != 512 && t != 1024)
            return fail(h, GP_E_ARG, "opts.batch_rows_t and batch_cols_t must be 0, 256, 512 or 1024");
    if (o.var_wave_rows < -1 || o.var_wave_rows > 1) return fail(h, GP_E_ARG, "opts.var_wave_rows must be -1, 0 or 1");
    if (o.var_item_rows != 0 && (o.var_item_rows < 16 || o.var_item_rows > 1024))
        return fail(h, GP_E_ARG, "opts.var_item_rows must be 0 or in 16..1024");
    if (o.batch_gemm_depth < 0 || o.batch_gemm_depth > 2)
        return fail(h, GP_E_ARG, "opts.batch_gemm_depth must be 0, 1 or 2");
    if (o.batch_gemm_tile != 0 && o.batch_gemm_tile != 64 && o.batch_gemm_tile != 128 && o.batch_gemm_tile != 256)
        return fail(h, GP_E_ARG, "opts.batch_gemm_tile must be 0, 64, 128 or 256");
    if (o.lookahead < 0) return fail(h, GP_E_ARG, "opts.lookahead must be >= 0");
    if ((o.batch_gemm_tile == 256 || o.batch_gemm_tile == 64) && o.batch_gemm_depth == 2)
        return fail(h, GP_E_ARG, "opts.batch_gemm_depth = 2 is for 128 x 128 GEMM tiles");
    return GP_OK_TOL;
}

// ---------------------------------------------------------------------------
// fused-kernel configurations
// ---------------------------------------------------------------------------
// (threads, column chunks per thread, rows per block); columns covered by one
// workgroup = T * CPT * VEC.
// (threads, column chunks per thread, rows per block, register buffers);
// columns covered by one workgroup = T * CPT * VEC.
// Shapes 11 and 12 keep the partial w in LDS (1024 threads, no spills).
struct FusedCfg { int T, CPT, RB, NB; };
static const FusedCfg kFusedCfgs[] = {
    {256, 1, 4, 2}, {256, 2, 4, 2}, {256, 4, 2, 2}, {512, 4, 2, 2}, {512, 8, 1, 2}, {1024, 8, 1, 2},
    {256, 4, 1, 3}, {512, 4, 1, 3}, {512, 8, 1, 3}, {1024, 4, 1, 3}, {1024, 4, 1, 2}, {1024, 2, 1, 3},
};
constexpr int kNumFusedCfgs = sizeof(kFusedCfgs) / sizeof(kFusedCfgs[0]);

int esize(gp_dtype dt) { return dt == GP_F64 ? 8 : dt == GP_F32 ? 4 : 2; }

// Pick the smallest configuration whose workgroup covers all p columns.
int pick_fused_cfg(gp_dtype dt, int64_t p, int want) {
    const int vec = 16 / esize(dt);
    if (want > 0 && want <= kNumFusedCfgs) {
        const FusedCfg& c = kFusedCfgs[want - 1];
        return (int64_t)c.T * c.CPT * vec >= p ? want - 1 : -1;
    }
    // automatic: at most 512 threads and 32 columns per thread.  Wider
    // one-pass shapes exceed the register budget (1024 threads: 128 per
    // lane; 64 bf16 columns per thread) and measured 1.3-6x slower than the
    // pass over column panels that takes over beyond them
    for (int i = 0; i < 6; ++i) {
        const FusedCfg& c = kFusedCfgs[i];
        if (c.T > 512 || c.CPT * vec > 32) break;
        if ((int64_t)c.T * c.CPT * vec >= p) return i;
    }
    return -1;
}

int64_t pick_fused_grid(int64_t n, int64_t p, gp_dtype dt, int want) {
    if (want > 0) return std::min<int64_t>(want, n);
    // one workgroup per CU for large problems; fewer for small ones so that
    // the partial vectors stay small next to K
    const double kbytes = (double)n * (double)p * esize(dt);
    int64_t g = kbytes >= 32e6 ? 256 : kbytes >= 4e6 ? 128 : 64;
    g = std::min<int64_t>(g, std::max<int64_t>(1, n / 2));
    return std::max<int64_t>(1, std::min(g, n));
}


template <typename TK, typename ACC, int T, int CPT, int RB, int NB, bool AL, bool WL>
void launch_fused_one(hipStream_t s, int64_t G, const FusedArgs& a) {
    if (a.ev0)   // start and stop stamped by the dispatch itself (no separate marker packets)
        hipExtLaunchKernelGGL((k_fused<TK, ACC, T, CPT, RB, NB, AL, WL>), dim3((unsigned)G), dim3(T), 0, s, a.ev0,
                              a.ev1, 0, a.st, (const TK*)a.K, a.n, a.p, a.ldk, a.rows, a.v, a.vsub, a.g, a.ysub,
                              a.rvec, a.tout, (ACC*)a.wpart, a.ldw, a.spart, a.interleave, a.v32);
    else
        hipLaunchKernelGGL((k_fused<TK, ACC, T, CPT, RB, NB, AL, WL>), dim3((unsigned)G), dim3(T), 0, s, a.st,
                           (const TK*)a.K, a.n, a.p, a.ldk, a.rows, a.v, a.vsub, a.g, a.ysub, a.rvec, a.tout,
                           (ACC*)a.wpart, a.ldw, a.spart, a.interleave, a.v32);
}

template <typename TK, typename ACC, int T, int CPT, int RB, int NB, bool WL = false>
void launch_fused_t(bool aligned, hipStream_t s, int64_t G, const FusedArgs& a) {
    if (aligned) launch_fused_one<TK, ACC, T, CPT, RB, NB, true, WL>(s, G, a);
    else launch_fused_one<TK, ACC, T, CPT, RB, NB, false, WL>(s, G, a);
}

template <typename TK, typename ACC>
void launch_fused_dt(int cfg, bool aligned, hipStream_t s, int64_t G, const FusedArgs& a) {
#define GPL1_FUSED_CASE(i, T, C, R, B) \
    case i: launch_fused_t<TK, ACC, T, C, R, B>(aligned, s, G, a); break;
    switch (cfg) {
        GPL1_FUSED_CASE(0, 256, 1, 4, 2)
        GPL1_FUSED_CASE(1, 256, 2, 4, 2)
        GPL1_FUSED_CASE(2, 256, 4, 2, 2)
        GPL1_FUSED_CASE(3, 512, 4, 2, 2)
        GPL1_FUSED_CASE(4, 512, 8, 1, 2)
        GPL1_FUSED_CASE(5, 1024, 8, 1, 2)
        GPL1_FUSED_CASE(6, 256, 4, 1, 3)
        GPL1_FUSED_CASE(7, 512, 4, 1, 3)
        GPL1_FUSED_CASE(8, 512, 8, 1, 3)
        GPL1_FUSED_CASE(9, 1024, 4, 1, 3)
        case 10: launch_fused_t<TK, ACC, 1024, 4, 1, 2, true>(aligned, s, G, a); break;
        case 11: launch_fused_t<TK, ACC, 1024, 2, 1, 3, true>(aligned, s, G, a); break;
    }
#undef GPL1_FUSED_CASE
}

// The two launches of a wide pass (grid: slabs x panels).  With timing
// events, the first launch stamps the start and the second the end.
template <typename TK, typename ACC, bool AL>
void launch_wide_one(hipStream_t s, int64_t G, const FusedArgs& a) {
    constexpr int T = WIDE_T, C = wide_cpt<TK>(), R = WIDE_RB;
    const dim3 grid((unsigned)G, (unsigned)a.np);
    hipExtLaunchKernelGGL((k_wide_t<TK, ACC, T, C, R, AL>), grid, dim3(T), 0, s, a.ev0, nullptr, 0, a.st,
                          (const TK*)a.K, a.n, a.p, a.ldk, a.rows, a.v, a.vsub, a.g, a.v32, a.tpart);
    hipExtLaunchKernelGGL((k_wide_w<TK, ACC, T, C, R, AL>), grid, dim3(T), 0, s, nullptr, a.ev1, 0, a.st,
                          (const TK*)a.K, a.n, a.p, a.ldk, a.rows, a.np, (const double*)a.tpart, a.v, a.vsub, a.g,
                          a.ysub, a.rvec, a.tout, (ACC*)a.wpart, a.ldw, a.spart);
}
template <typename TK, typename ACC>
void launch_wide(bool aligned, hipStream_t s, int64_t G, const FusedArgs& a) {
    if (aligned) launch_wide_one<TK, ACC, true>(s, G, a);
    else launch_wide_one<TK, ACC, false>(s, G, a);
}

int64_t wide_panel_cols(gp_dtype dt) {
    return dt == GP_F64 ? wide_panel<double>() : dt == GP_F32 ? wide_panel<float>() : wide_panel<bf16_t>();
}

void launch_fused(gp_dtype dt, int cfg, bool aligned, hipStream_t s, int64_t G, const FusedArgs& a) {
    if (cfg == kCfgWide) {
        if (dt == GP_F64) launch_wide<double, double>(aligned, s, G, a);
        else if (dt == GP_F32) launch_wide<float, float>(aligned, s, G, a);
        else launch_wide<bf16_t, float>(aligned, s, G, a);
        return;
    }
    if (dt == GP_F64) launch_fused_dt<double, double>(cfg, aligned, s, G, a);
    else if (dt == GP_F32) launch_fused_dt<float, float>(cfg, aligned, s, G, a);
    else launch_fused_dt<bf16_t, float>(cfg, aligned, s, G, a);
}

// Shape of the single-workgroup projection: threads T and register slots per
// thread (pairs of neighbours, so at least 2; 0 streams through vbuf).
// Measured (kernel durations of one process, p = 2048 to 16384): eight waves
// up to p = 8192, where fewer waves make each threshold pass's workgroup
// reduction cheaper; sixteen waves above, where the single workgroup's loads
// of x and g and its stores of h and d dominate.  x and g stay in registers
// while T * slots <= 16384.
struct ProjShape { int T, vpt; };

ProjShape proj_shape(int64_t p) {
    if (p <= 512 * 16) {
        const int64_t per = (p + 511) / 512;
        int v = 2;
        while (v < per) v *= 2;
        return {512, v};
    }
    if (p <= 1024 * 16) return {1024, 16};
    if (p <= 1024 * 22) return {1024, 22};
    return {1024, 0};
}

void launch_proj(hipStream_t s, GPState* st, int mode, int64_t p, double* x, const double* g, double* dout,
                 const double* upart, int GU, double* vbuf, float* d32) {
    const ProjShape sh = proj_shape(p);
    switch (sh.T * 100 + sh.vpt) {
#define GPL1_PROJ_CASE(T, V) \
    case T * 100 + V: \
        hipLaunchKernelGGL((k_proj<V, T>), dim3(1), dim3(T), 0, s, st, mode, p, x, g, dout, upart, GU, vbuf, d32); \
        break;
        GPL1_PROJ_CASE(512, 2)
        GPL1_PROJ_CASE(512, 4)
        GPL1_PROJ_CASE(512, 8)
        GPL1_PROJ_CASE(512, 16)      // p in (4096, 8192]
        GPL1_PROJ_CASE(1024, 16)     // p in (8192, 16384]
        GPL1_PROJ_CASE(1024, 22)
        GPL1_PROJ_CASE(1024, 0)
#undef GPL1_PROJ_CASE
    }
}

void launch_update(gp_dtype dt, hipStream_t s, GPState* st, int mode, const double* spart, int GF,
                   const void* wpart, int64_t ldw, int64_t p, int64_t n, double* x, double* g,
                   double* r, const double* tq, double* upart) {
    const int nbp = (int)((p + UPD_COLS - 1) / UPD_COLS);
    const int nbn = (int)((n + UPD_ROWS - 1) / UPD_ROWS);
    if (dt == GP_F64)
        hipLaunchKernelGGL(k_update<double>, dim3(nbp + nbn), dim3(UPD_T), 0, s, st, mode, spart, GF,
                           (const double*)wpart, ldw, p, n, nbp, x, g, r, tq, upart);
    else
        hipLaunchKernelGGL(k_update<float>, dim3(nbp + nbn), dim3(UPD_T), 0, s, st, mode, spart, GF,
                           (const float*)wpart, ldw, p, n, nbp, x, g, r, tq, upart);
}

template <typename TV>
void launch_to_f64(hipStream_t s, const void* in, double* out, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f64<TV>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const TV*)in, out, n);
}
template <typename TV>
void launch_from_f64(hipStream_t s, const double* in, void* out, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_from_f64<TV>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, (TV*)out, n);
}

// ---------------------------------------------------------------------------
// one problem
// ---------------------------------------------------------------------------
Plan plan_single(gp_dtype dt, int64_t n, int64_t p, const gp_opts& o) {
    Plan P{};
    // the two-launch pass over column panels: asked for (GP_FUSED_PANELS), or
    // automatic beyond the widest one-pass configuration
    const bool panels = o.fused_cfg == GP_FUSED_PANELS;
    P.cfg = panels ? -1 : pick_fused_cfg(dt, p, o.fused_cfg);
    P.np = 0;
    if (panels || (P.cfg < 0 && o.fused_cfg <= 0)) {
        const int64_t np = (p + wide_panel_cols(dt) - 1) / wide_panel_cols(dt);
        if (np <= 65535) {   // the panels are the grid's second dimension
            P.cfg = kCfgWide;
            P.np = (int)np;
        }
    }
    P.G = pick_fused_grid(n, p, dt, o.fused_grid);
    P.rows = (n + P.G - 1) / P.G;
    P.G = (n + P.rows - 1) / P.rows;
    P.ldw = (p + 63) / 64 * 64;
    P.nbp = (int)((p + UPD_COLS - 1) / UPD_COLS);
    P.GU = P.nbp + (int)((n + UPD_ROWS - 1) / UPD_ROWS);
    const int wsz = dt == GP_F64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += (bytes + 255) / 256 * 256; return o2; };
    P.o_state = take(sizeof(GPState));
    P.o_x = take(sizeof(double) * p);
    P.o_g = take(sizeof(double) * p);
    P.o_d = take(sizeof(double) * p);
    P.o_vbuf = take(sizeof(double) * p);
    P.o_d32 = take(sizeof(float) * p);
    P.o_r = take(sizeof(double) * n);
    P.o_q = take(sizeof(double) * n);
    P.o_y = take(sizeof(double) * n);
    P.o_spart = take(sizeof(double) * SPART * P.G);
    P.o_upart = take(sizeof(double) * 4 * P.GU);
    P.o_wpart = take((size_t)wsz * P.ldw * P.G);
    P.nvitems = (int)((n + VR_ROWS - 1) / VR_ROWS);
    P.o_vprob = take(sizeof(VerProb));
    P.o_vitem = take(sizeof(VerItem) * P.nvitems);
    P.o_vpart = take(sizeof(double) * P.nvitems);
    P.o_vidx = take(sizeof(int32_t) * 4);
    P.o_tpart = take(sizeof(double) * (size_t)P.np * n);
    P.bytes = off;
    return P;
}

void launch_verify_rows(gp_dtype dt, hipStream_t s, int nitems, const VerProb* vp, const VerItem* items,
                        double* part) {
    if (nitems <= 0) return;
    if (dt == GP_F64)
        hipLaunchKernelGGL(k_verify_rows<double>, dim3((unsigned)nitems), dim3(VR_T), 0, s, vp, items, part);
    else if (dt == GP_F32)
        hipLaunchKernelGGL(k_verify_rows<float>, dim3((unsigned)nitems), dim3(VR_T), 0, s, vp, items, part);
    else
        hipLaunchKernelGGL(k_verify_rows<bf16_t>, dim3((unsigned)nitems), dim3(VR_T), 0, s, vp, items, part);
}

}  // namespace gpl1

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void gp_opts_default(gp_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->M = 1;
    o->theta = 0.5;
    o->beta = 1e-4;
    o->alpha_min = 1e-10;
    o->alpha_max = 1e10;
    o->tau1 = 0.5;
    o->M_alpha = 2;
    o->max_iter = 100000;
    o->f_target = -1.0;
    o->refresh_every = 0;
    o->backtrack_cap = 60;
    o->chunk = 64;
    o->fused_cfg = 0;
    o->fused_grid = 0;
    o->profile = 0;
    o->fused_interleave = 0;
    o->f_targets = nullptr;
    o->x0_fallback = 0;
    o->graph = 0;
    o->batch_splitk = 0;
    o->batch_rows_t = 0;
    o->batch_cols_t = 0;
    o->var_item_rows = 0;
    o->batch_gemm_depth = 0;
    o->batch_gemm_tile = 0;
    o->lookahead = 2;
    o->var_wave_rows = 0;
}

int gp_create(gp_handle* out, int device) {
    if (!out) return GP_E_ARG;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device < 0 || device >= count) return GP_E_ARG;
    gp_handle h = new (std::nothrow) gp_handle_s();
    if (!h) return GP_E_NOMEM;
    h->device = device;
    e = hipSetDevice(device);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->host_state, sizeof(GPState), hipHostMallocDefault);
    // the progress word: coherent, so the device's system-scope stores reach
    // the host's loads without a synchronisation
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&h->progress, 64, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&h->progress_dev, h->progress, 0);
    if (e != hipSuccess) {
        if (h->progress) (void)hipHostFree(h->progress);
        if (h->host_state) (void)hipHostFree(h->host_state);
        delete h;
        return GP_E_HIP;
    }
    // the allocation-free solve's scratch: its address on this device (the
    // device is current here)
    if (setup_scratch(device) != GP_OK_TOL) {
        (void)hipHostFree(h->progress);
        (void)hipHostFree(h->host_state);
        delete h;
        return GP_E_HIP;
    }
    *out = h;
    return GP_OK_TOL;
}

int gp_destroy(gp_handle h) {
    if (!h) return GP_OK_TOL;
    (void)hipSetDevice(h->device);
    if (h->ws) (void)hipFree(h->ws);
    if (h->host_state) (void)hipHostFree(h->host_state);
    if (h->progress) (void)hipHostFree(h->progress);
    if (h->pin) (void)hipHostFree(h->pin);
    for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->gexec_b) (void)hipGraphExecDestroy(h->gexec_b);
    if (h->gevent) (void)hipEventDestroy(h->gevent);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    delete h;
    return GP_OK_TOL;
}

const char* gp_last_error(gp_handle h) {
    if (!h) return "null handle";
    return h->err.c_str();
}

int gp_l1_project(gp_handle h, gp_dtype vdtype, const void* v, int64_t p, double rho, void* h_out,
                  double* mu_out, void* stream) {
    if (!h) return GP_E_ARG;
    h->err.clear();
    if (vdtype != GP_F64 && vdtype != GP_F32) return fail(h, GP_E_ARG, "projection vectors must be GP_F64 or GP_F32");
    if (p < 0) return fail(h, GP_E_ARG, "p must be >= 0");
    if (!(rho >= 0.0) || !std::isfinite(rho)) return fail(h, GP_E_ARG, "rho must be finite and >= 0");
    if (p == 0) { if (mu_out) *mu_out = 0.0; return GP_OK_TOL; }
    if (!v || !h_out) return fail(h, GP_E_ARG, "null vector pointer");
    if (p > (int64_t)1 << 31) return fail(h, GP_E_UNSUPPORTED, "p too large");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += (bytes + 255) / 256 * 256; return o2; };
    size_t o_state = take(sizeof(GPState)), o_x = take(8 * p), o_h = take(8 * p), o_vb = take(8 * p);
    int rc = ensure_workspace(h, off);
    if (rc) return rc;
    char* ws = (char*)h->ws;
    GPState* st = (GPState*)(ws + o_state);
    double* x = (double*)(ws + o_x);
    double* hv = (double*)(ws + o_h);
    double* vb = (double*)(ws + o_vb);
    gp_opts o;
    gp_opts_default(&o);
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, make_params(o, rho, 0.0));
    if (vdtype == GP_F64) launch_to_f64<double>(s, v, x, p);
    else launch_to_f64<float>(s, v, x, p);
    launch_proj(s, st, PM_PLAIN, p, x, nullptr, hv, nullptr, 0, vb, nullptr);
    if (vdtype == GP_F64) launch_from_f64<double>(s, hv, h_out, p);
    else launch_from_f64<float>(s, hv, h_out, p);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "projection launch");
    if (mu_out) {
        e = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "projection sync");
        if (h->host_state->status == ST_NONFINITE) return fail(h, GP_E_NONFINITE, "non-finite input vector");
        *mu_out = h->host_state->mu;
    }
    return GP_OK_TOL;
}

}  // extern "C"

namespace gpl1 {

// One problem.  `fixed_ws` NULL: the handle's workspace, grown on demand;
// otherwise the caller-provided device buffer of `fixed_bytes` (nothing is
// allocated, and shapes whose workspace does not fit are refused).
static int solve_single(gp_handle h, gp_dtype kdtype, const void* K, int64_t n, int64_t p, int64_t ldk,
                        const void* y, double rho, const void* x0, double tol, void* x_out, const gp_opts* opts,
                        gp_result* res, void* stream, void* fixed_ws, size_t fixed_bytes) {
    if (!h) return GP_E_ARG;
    h->err.clear();
    if (!res) return fail(h, GP_E_ARG, "res must not be NULL");
    std::memset(res, 0, sizeof(*res));
    res->status = GP_E_ARG;
    gp_opts o;
    if (opts) o = *opts; else gp_opts_default(&o);
    if (kdtype != GP_F64 && kdtype != GP_F32 && kdtype != GP_BF16) return fail(h, GP_E_ARG, "bad dtype");
    if (n <= 0 || p <= 0) return fail(h, GP_E_ARG, "n and p must be positive");
    if (ldk < p) return fail(h, GP_E_ARG, "ldk must be >= p");
    if (!(rho >= 0.0) || !std::isfinite(rho)) return fail(h, GP_E_ARG, "rho must be finite and >= 0");
    if (!(tol >= 0.0)) return fail(h, GP_E_ARG, "tol must be >= 0");
    if (!K || !y || !x_out) return fail(h, GP_E_ARG, "null pointer argument");
    int rc = check_opts(h, o);
    if (rc) return rc;
    if (n > ((int64_t)1 << 31) || p > ((int64_t)1 << 31)) return fail(h, GP_E_UNSUPPORTED, "n or p too large");
    Plan P = plan_single(kdtype, n, p, o);
    if (P.cfg < 0)
        return fail(h, GP_E_UNSUPPORTED, "p = " + std::to_string(p) + " exceeds the fused kernel's column capacity");
    if (fixed_ws) {
        if (o.graph || o.profile)
            return fail(h, GP_E_ARG, "the allocation-free solve takes neither opts.graph nor opts.profile");
        if (P.bytes > fixed_bytes)
            return fail(h, GP_E_UNSUPPORTED, "n = " + std::to_string(n) + ", p = " + std::to_string(p) +
                                                 " needs " + std::to_string(P.bytes) +
                                                 " bytes of workspace; the fixed scratch holds " +
                                                 std::to_string(fixed_bytes));
    }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    if (!fixed_ws) {
        rc = ensure_workspace(h, P.bytes);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    if (o.graph && (rc = graph_stream(h, (hipStream_t)stream, &s))) return rc;
    char* ws = fixed_ws ? (char*)fixed_ws : (char*)h->ws;
    GPState* st = (GPState*)(ws + P.o_state);
    double* x = (double*)(ws + P.o_x);
    double* g = (double*)(ws + P.o_g);
    double* d = (double*)(ws + P.o_d);
    double* vb = (double*)(ws + P.o_vbuf);
    // float copy of d for the fused pass (its products are float for FP32 and bf16 K)
    float* d32 = kdtype == GP_F64 ? nullptr : (float*)(ws + P.o_d32);
    double* r = (double*)(ws + P.o_r);
    double* q = (double*)(ws + P.o_q);
    double* y64 = (double*)(ws + P.o_y);
    double* spart = (double*)(ws + P.o_spart);
    double* upart = (double*)(ws + P.o_upart);
    void* wpart = ws + P.o_wpart;
    const int vec = 16 / esize(kdtype);
    // the fused pass's branch-free loads need whole chunks: rows 16-byte
    // aligned and p a multiple of the chunk
    const bool aligned = (ldk % vec == 0) && (p % vec == 0) && (((uintptr_t)K) % 16 == 0);
    const bool f64v = kdtype == GP_F64;

    // lookahead: the update kernel posts its progress to the handle's
    // host-mapped word, cleared here (the handle's last solve has ended with
    // a synchronising poll, so no launch of it can still write the word)
    const bool ahead = o.lookahead > 0 && !o.graph;
    if (ahead) __atomic_store_n(h->progress, 0u, __ATOMIC_RELEASE);
    {
        GPParams prm = make_params(o, rho, tol);
        if (ahead) prm.progress = h->progress_dev;
        if (o.trace) {
            prm.trace = o.trace;
            prm.trace_cap = o.trace_cap;
        }
        const unsigned sg = (unsigned)((std::max(n, p) + 255) / 256);
        if (f64v)
            hipLaunchKernelGGL(k_setup<double>, dim3(sg), dim3(256), 0, s, st, prm,
                               (const double*)y, y64, n, (const double*)x0, x, p);
        else
            hipLaunchKernelGGL(k_setup<float>, dim3(sg), dim3(256), 0, s, st, prm,
                               (const float*)y, y64, n, (const float*)x0, x, p);
    }
    if (x0) launch_proj(s, st, PM_INIT_X0, p, x, nullptr, nullptr, nullptr, 0, vb, nullptr);
    // r = K x - y, g = 2 K^T r, f = ||r||^2
    // an iteration stores no h: the projection leaves (alpha, m, t, mode) in
    // the state and the float copy of d, and the fused and update kernels
    // recompute h from x and g; d only parks P(x0) during the x0 check
    const int il = o.fused_interleave;
    FusedArgs fa_refresh{st, K, n, p, ldk, P.rows, x, nullptr, nullptr, y64, nullptr, q, wpart, P.ldw, spart, il,
                         nullptr};
    // iteration: h is recomputed from x and g inside the fused kernel (v NULL)
    FusedArgs fa_iter{st, K, n, p, ldk, P.rows, nullptr, x, g, nullptr, r, q, wpart, P.ldw, spart, il, d32};
    fa_refresh.tpart = fa_iter.tpart = (double*)(ws + P.o_tpart);
    fa_refresh.np = fa_iter.np = P.np;
    auto refresh = [&]() {
        launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_refresh);
        launch_update(kdtype, s, st, UM_REFRESH, spart, (int)P.G, wpart, P.ldw, p, n, x, g, r, q, upart);
    };
    int x0_rejected = 0;
    if (x0 && o.x0_fallback) {
        // f(0) = ||y||^2 from a residual pass at x = 0 (P(x0) parked in d),
        // then f(P(x0)); x0 is kept only if it is strictly better
        e = hipMemcpyAsync(d, x, 8 * p, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(x, 0, 8 * p, s);
        if (e != hipSuccess) return hip_fail(h, e, "x0 fallback");
        refresh();
        e = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "x0 fallback");
        const double f0 = h->host_state->f_new;     // a refresh stages f until the next projection commits it
        e = hipMemcpyAsync(x, d, 8 * p, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(h, e, "x0 fallback");
        refresh();
        e = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "x0 fallback");
        if (!(h->host_state->f_new < f0)) {
            x0_rejected = 1;
            e = hipMemsetAsync(x, 0, 8 * p, s);
            if (e != hipSuccess) return hip_fail(h, e, "x0 fallback");
            refresh();
        }
    } else {
        refresh();
    }
    launch_proj(s, st, PM_ALPHA0, p, x, g, nullptr, nullptr, 0, vb, nullptr);
    // target check set-up: rows of K against x (narrowed as returned) and y
    const bool check_target = o.f_target >= 0.0;
    VerProb* vprob = (VerProb*)(ws + P.o_vprob);
    VerItem* vitems = (VerItem*)(ws + P.o_vitem);
    double* vpart = (double*)(ws + P.o_vpart);
    int32_t* vidx = (int32_t*)(ws + P.o_vidx);
    if (check_target) {
        const int esz_k = esize(kdtype);
        const VerProb vp{K, ldk, n, p, x, y64, f64v ? 0 : 1,
                         ((ldk * esz_k) % 16 == 0 && ((uintptr_t)K) % 16 == 0) ? 1 : 0};
        hipLaunchKernelGGL(k_verify_setup_single, dim3((unsigned)((P.nvitems + 255) / 256)), dim3(256), 0, s, vprob,
                           vitems, vidx, P.nvitems, vp);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "init launch");

    // graph mode: chunks of gch iterations starting at multiples of gch, each
    // ending with the refresh that the plain schedule puts there
    const int gch = o.refresh_every > 0 ? o.refresh_every : o.chunk;
    auto graph_chunk = [&]() -> int {
        const std::vector<int64_t> key = {(int64_t)kdtype, (int64_t)(uintptr_t)K, n, p, ldk, P.cfg, P.G,
                                          aligned ? 1 : 0, il, (int64_t)(uintptr_t)h->ws, gch,
                                          o.refresh_every, (int64_t)(uintptr_t)s};
        if (!h->gexec || h->gkey != key) {
            if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
            const int crc = capture_graph(h, s, &h->gexec, [&]() {
                for (int k = 0; k < gch; ++k) {
                    launch_proj(s, st, PM_ITER, p, x, g, nullptr, upart, P.GU, vb, d32);
                    launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_iter);
                    launch_update(kdtype, s, st, UM_ITER, spart, (int)P.G, wpart, P.ldw, p, n, x, g, r, q, upart);
                }
                if (o.refresh_every > 0) refresh();
            });
            if (crc) return crc;
            h->gkey = key;
        }
        const hipError_t le = hipGraphLaunch(h->gexec, s);
        return le == hipSuccess ? 0 : hip_fail(h, le, "graph launch");
    };

    // status poll after a chunk: the finishing kernel goes first, so a poll
    // that sees the solve stopped already holds its result (and x_out)
    auto poll = [&](bool last) -> int {
        if (f64v)
            hipLaunchKernelGGL(k_finish<double>, dim3(1), dim3(PROJ_T), 0, s, st, x, g, p, last ? 1 : 0,
                               (double*)x_out);
        else
            hipLaunchKernelGGL(k_finish<float>, dim3(1), dim3(PROJ_T), 0, s, st, x, g, p, last ? 1 : 0,
                               (float*)x_out);
        hipError_t pe = hipGetLastError();
        if (pe == hipSuccess) pe = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
        if (pe == hipSuccess) pe = hipStreamSynchronize(s);
        return pe == hipSuccess ? 0 : hip_fail(h, pe, "status poll");
    };
    // after a poll that found the solve stopped at its target: recompute f in
    // double and keep the stop (0) or reopen the solve (1); < 0: an error
    auto check = [&]() -> int {
        if (!check_target || !target_checkable(h->host_state->status) || h->host_state->tcheck) return 0;
        launch_verify_rows(kdtype, s, P.nvitems, vprob, vitems, vpart);
        hipLaunchKernelGGL(k_verify_decide, dim3(1), dim3(64), 0, s, st, vidx, vidx + 1, 1, vpart, 0);
        hipError_t ce = hipGetLastError();
        if (ce == hipSuccess) ce = hipMemcpyAsync(h->host_state, st, sizeof(GPState), hipMemcpyDeviceToHost, s);
        if (ce == hipSuccess) ce = hipStreamSynchronize(s);
        if (ce != hipSuccess) return hip_fail(h, ce, "target check");
        return h->host_state->done ? 0 : 1;
    };
    // one iteration's launches: projection (with the steplength rule), fused
    // K / K^T pass, update, and the residual refresh where one falls due
    auto enqueue_iteration = [&](int i) {
        launch_proj(s, st, PM_ITER, p, x, g, nullptr, upart, P.GU, vb, d32);
        // every profile-th iteration's fused launch is bracketed by events
        if (o.profile > 0 && i % o.profile == 0) {
            FusedArgs fa = fa_iter;
            fa.ev0 = prof_event(h);
            fa.ev1 = fa.ev0 ? prof_event(h) : nullptr;
            if (fa.ev0 && !fa.ev1) { --h->ev_used; fa.ev0 = nullptr; }   // keep the pairs aligned
            launch_fused(kdtype, P.cfg, aligned, s, P.G, fa);
        } else {
            launch_fused(kdtype, P.cfg, aligned, s, P.G, fa_iter);
        }
        launch_update(kdtype, s, st, UM_ITER, spart, (int)P.G, wpart, P.ldw, p, n, x, g, r, q, upart);
        if (o.refresh_every > 0 && (i + 1) % o.refresh_every == 0 && i + 1 < o.max_iter) refresh();
    };
    // lookahead: wait until the device has completed `need` updates (0), has
    // posted a stop (1), or has run out of launches without either (2: a
    // stop that the update kernel does not post, or a device faster than the
    // host); < 0 is an error
    auto wait_progress = [&](int need) -> int {
        auto last = std::chrono::steady_clock::now();
        for (;;) {
            const uint32_t w = __atomic_load_n(h->progress, __ATOMIC_ACQUIRE);
            if (w & 0x80000000u) return 1;
            if ((int)(w & 0x7fffffffu) >= need) return 0;
            const auto now = std::chrono::steady_clock::now();
            // the stream is queried only after a millisecond without news: a
            // query can enqueue a marker between the kernels
            if (now - last > std::chrono::milliseconds(1)) {
                last = now;
                const hipError_t q = hipStreamQuery(s);
                if (q == hipSuccess) return 2;
                if (q != hipErrorNotReady) return hip_fail(h, q, "progress wait");
            }
            __builtin_ia32_pause();
        }
    };
    bool finished = false;
    int it = 0;
    while (it < o.max_iter) {
        if (ahead) {
            for (; it < o.max_iter; ++it) {
                const int wr = wait_progress(it - o.lookahead);
                if (wr < 0) return wr;
                if (wr == 1) break;
                if (wr == 2) {
                    // the device is idle and posted no stop: read its state
                    if ((rc = poll(false))) return rc;
                    if (h->host_state->done) break;
                }
                enqueue_iteration(it);
            }
            e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(h, e, "iteration launch");
            if ((rc = poll(it >= o.max_iter))) return rc;
            if (h->host_state->done) {
                const int re = check();
                if (re < 0) return re;
                if (re) {
                    // reopened: the stream is idle, so the word can be reset
                    it = h->host_state->k;
                    __atomic_store_n(h->progress, (uint32_t)it, __ATOMIC_RELEASE);
                    continue;
                }
                finished = true;
                break;
            }
            // a posted stop that the state does not show: pace by the updates again
            __atomic_store_n(h->progress, (uint32_t)h->host_state->k, __ATOMIC_RELEASE);
            continue;
        }
        if (o.graph && it % gch == 0 && it + gch < o.max_iter) {
            rc = graph_chunk();
            if (rc) return rc;
            it += gch;
            if ((rc = poll(false))) return rc;
            if (h->host_state->done) {
                const int re = check();
                if (re < 0) return re;
                if (re) { it = h->host_state->k; continue; }
                finished = true;
                break;
            }
            continue;
        }
        const int end = o.graph ? std::min(o.max_iter, (it / gch + 1) * gch) : std::min(o.max_iter, it + o.chunk);
        for (; it < end; ++it) enqueue_iteration(it);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "iteration launch");
        if ((rc = poll(it >= o.max_iter))) return rc;
        if (h->host_state->done) {
            const int re = check();
            if (re < 0) return re;
            if (re) { it = h->host_state->k; continue; }
            finished = true;
            break;
        }
    }
    if (!finished && (rc = poll(true))) return rc;
    // the budget is spent: check the last stop; a target stop reopened here
    // has no iterations left and ends at the budget
    for (int guard = 0; guard < 2; ++guard) {
        const int re = check();
        if (re < 0) return re;
        if (re == 0) break;
        if ((rc = poll(true))) return rc;
    }
    fill_result(*h->host_state, res);
    res->x0_rejected = x0_rejected;
    if (o.profile) {
        // fused launches that did work: one per accepted update, plus the one
        // whose direction was found stationary or failed the line search
        const int live = res->iters + ((res->status == GP_STATIONARY || res->status == GP_BACKTRACK_LIMIT) ? 1 : 0);
        res->t_fused_ms = prof_collect(h, (live + o.profile - 1) / o.profile, &res->n_fused);
    }
    if (res->status < 0) return fail(h, res->status, "solve ended with a non-finite value");
    return res->status;
}

}  // namespace gpl1

extern "C" {

int gp_l1_solve(gp_handle h, gp_dtype kdtype, const void* K, int64_t n, int64_t p, int64_t ldk, const void* y,
                double rho, const void* x0, double tol, void* x_out, const gp_opts* opts, gp_result* res,
                void* stream) {
    return solve_single(h, kdtype, K, n, p, ldk, y, rho, x0, tol, x_out, opts, res, stream, nullptr, 0);
}

int gp_l1_solve_noalloc(gp_handle h, gp_dtype kdtype, const void* K, int64_t n, int64_t p, int64_t ldk,
                        const void* y, double rho, const void* x0, double tol, void* x_out, const gp_opts* opts,
                        gp_result* res, void* stream) {
    if (!h) return GP_E_ARG;
    void* ptr = scratch_ptr(h->device);
    if (!ptr) {
        if (res) { std::memset(res, 0, sizeof(*res)); res->status = GP_E_HIP; }
        return fail(h, GP_E_HIP, "the fixed scratch of this device has no address (gp_create did not set it up)");
    }
    return solve_single(h, kdtype, K, n, p, ldk, y, rho, x0, tol, x_out, opts, res, stream, ptr,
                        (size_t)GP_NOALLOC_SCRATCH_BYTES);
}

}  // extern "C"

namespace gpl1 {
void fill_result(const GPState& s, gp_result* res) {
    res->status = s.status;
    res->iters = s.k;
    res->backtracks = s.backtracks;
    res->projected_x0 = s.projected;
    res->f = s.f;
    res->rel_change = s.rel;
    res->lambda_est = s.gmax / 2.0;
    res->l1norm = s.l1;
    res->proj_passes = s.michelot_total;
    res->x0_rejected = s.x0_rejected;
    res->reopened = s.reopened;
}
}  // namespace gpl1
