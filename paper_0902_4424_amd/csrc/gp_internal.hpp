// Host-side internals shared by the API translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "gp_l1.h"
#include "gp_state.hpp"

struct gp_handle_s {
    int device = 0;
    std::string err;
    void* ws = nullptr;                  // device workspace, grows on demand
    size_t ws_bytes = 0;
    gpl1::GPState* host_state = nullptr; // pinned copy of a state for status reads
    uint32_t* progress = nullptr;        // host-mapped word the update kernel posts its progress to
    uint32_t* progress_dev = nullptr;    // its device address
    void* pin = nullptr;                 // pinned host buffer of the batched status polls, grows on demand
    size_t pin_bytes = 0;
    void* extra = nullptr;               // batched-solver resources
    std::vector<hipEvent_t> events;      // profiling: start/stop pairs of fused launches
    int ev_used = 0;
    // graph mode of the single-problem solver: a captured chunk of iterations,
    // kept while the launch arguments it was captured with stay the same
    hipStream_t gstream = nullptr;       // capture stream when the caller passes the null stream
    hipEvent_t gevent = nullptr;         // orders it with the caller's stream
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gkey;           // the arguments of the captured chunk
    hipGraphExec_t gexec_b = nullptr;    // the batched solvers' captured chunk (per call)
};

namespace gpl1 {

// Workspace layout and launch shapes of one problem.
struct Plan {
    int cfg;          // fused-kernel configuration index
    int64_t G;        // fused-kernel workgroups (row slabs)
    int64_t rows;     // rows per slab
    int64_t ldw;      // stride of the partial w vectors
    int nbp, GU;      // update kernel: column workgroups, all workgroups
    size_t o_state, o_x, o_g, o_d, o_vbuf, o_d32, o_r, o_q, o_y, o_spart, o_upart, o_wpart, bytes;
    // exact check of an objective target: problem descriptor, row items,
    // partial sums, the (one) checked problem and its item range
    size_t o_vprob, o_vitem, o_vpart, o_vidx;
    int nvitems;
    // wide problems: column panels (0 when one workgroup holds every column)
    // and the panels' partial dots (np * n)
    int np;
    size_t o_tpart;
};

// Arguments of one fused K / K^T launch (see k_fused).
struct FusedArgs {
    const GPState* st; const void* K; int64_t n, p, ldk, rows;
    const double *v, *vsub, *g, *ysub, *rvec; double* tout; void* wpart; int64_t ldw; double* spart;
    int interleave;
    const float* v32;   // float copy of the multiplied vector, or NULL
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // timing: recorded by the launch itself
    // wide problems (cfg == kCfgWide): np column panels and their partial dots
    double* tpart = nullptr;
    int np = 0;
};
// The fused configuration index of the two-launch pass over column panels.
constexpr int kCfgWide = 1000;
void launch_fused(gp_dtype dt, int cfg, bool aligned, hipStream_t s, int64_t G, const FusedArgs& a);
Plan plan_single(gp_dtype dt, int64_t n, int64_t p, const gp_opts& o);
int esize(gp_dtype dt);
struct VerProb;
struct VerItem;
void launch_verify_rows(gp_dtype dt, hipStream_t s, int nitems, const VerProb* vp, const VerItem* items,
                        double* part);

// Graph replay: the stream to capture on (the handle's own one, ordered
// after the caller's work, when the caller passes the null stream), and the
// capture of what `enqueue` launches into `exec` (replacing its old graph).
int graph_stream(gp_handle h, hipStream_t user, hipStream_t* out);
int capture_graph(gp_handle h, hipStream_t s, hipGraphExec_t* exec, const std::function<void()>& enqueue);

int fail(gp_handle h, int code, const std::string& msg);
int hip_fail(gp_handle h, hipError_t e, const char* where);
int ensure_workspace(gp_handle h, size_t bytes);
int ensure_pinned(gp_handle h, size_t bytes);
void fill_result(const GPState& s, gp_result* res);
void destroy_extra(gp_handle h);
const char* status_name(int s);
GPParams make_params(const gp_opts& o, double rho, double tol);
int check_opts(gp_handle h, const gp_opts& o);
// Batched shared-K solve on the matrix cores (bf16 K); GP_E_UNSUPPORTED means
// nothing was launched and the caller should use another path.
int solve_batched_shared_mfma(gp_handle h, gp_dtype kdtype, const void* K, int64_t n, int64_t p, int64_t ldk,
                              const void* Y, int64_t ldy, int64_t B, const double* rho, const void* X0,
                              int64_t ldx, double tol, void* X_out, const gp_opts& o, gp_result* res,
                              hipStream_t s);
// Independent problems in lockstep; GP_E_UNSUPPORTED means nothing was
// launched and the caller should solve them one at a time.
int solve_batched_var_lockstep(gp_handle h, gp_dtype kdtype, const gp_instance* inst, int64_t B, double tol,
                               const gp_opts& o, gp_result* res, hipStream_t s);
// Profiling helpers: record an event pair around a launch; sum at the end.
hipEvent_t prof_event(gp_handle h);
double prof_collect(gp_handle h, int live, int* pairs);

}  // namespace gpl1
