// Internal declarations of the PAM HIP library (gfx950). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "pam.h"

namespace pam {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);

#define PAM_CHECK_HIP(expr)                                                           \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            ::pam::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));      \
            return PAM_ERR_HIP;                                                       \
        }                                                                             \
    } while (0)

#define PAM_REQUIRE(cond, msg)                                                        \
    do {                                                                              \
        if (!(cond)) {                                                                \
            ::pam::set_error(msg);                                                    \
            return PAM_ERR_ARG;                                                       \
        }                                                                             \
    } while (0)

// ---------------------------------------------------------------- workspace
enum Buf {
    BUF_WT = 0,     // normalized design, transposed [n_sub][mpad][npad] (f64/f32/bf16)
    BUF_G,          // Gram incl. data row [n_sub][mpad][mpad] (f64 or f32)
    BUF_H,          // inverse of the active block, per subdomain (solve_h_elems) f64
    BUF_VEC,        // per-subdomain scratch of the blocked bordering (solve_scratch_elems) f64
    BUF_TABLE,      // small launch tables (per-subdomain parameters)
    BUF_R,          // indicator values [N_tot] f64
    BUF_MARK,       // ranking keys and indices of subdomains beyond the LDS sort
    BUF_EVAL,       // query binning workspace
    BUF_FLAGS,      // per-subdomain flags / counters
    BUF_CNN,        // network activations, packed weights, gradient partials
    BUF_TEAM,       // control words of the solve's workgroup teams
    BUF_AUX,        // staging of generated query points (Darcy coefficient)
    BUF_ROWSUM,     // Shepard denominators 1 / sum_m phi_jm of the fused Gram path [n_sub][npad] f32
    BUF_COUNT
};

struct Workspace {
    void *ptr[BUF_COUNT] = {};
    size_t bytes[BUF_COUNT] = {};
};

// Pinned staging buffer for small host tables; `done` marks the end of the
// previous upload so the buffer is not overwritten while a copy is pending.
struct Staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};

// Opt-in per-launch event timing (pam_timing_enable).
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> pool;                // free events
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double ms[PAM_TK_COUNT] = {};
    int64_t count[PAM_TK_COUNT] = {};
};

}  // namespace pam

namespace pam {
// Executable graphs of fit / refinement calls, keyed by everything that
// shapes their launches (pointers, sizes, options, workspace addresses).
struct GraphCache {
    struct Entry { uint64_t key; hipGraphExec_t exec; uint64_t used; };
    std::vector<Entry> entries;
    uint64_t clock = 0;
    hipStream_t capture = nullptr;         // private stream the calls are captured on
    bool on = true;                        // pam_graph_enable
    bool capturing = false;                // a capture is in progress (workspace frozen)
};
}  // namespace pam

struct pam_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    pam::Workspace ws;
    pam::Staging staging;
    pam::Timing timing;
    pam::GraphCache graphs;
    int32_t *sticky = nullptr;   // device [4]: [0] subdomains met with non-finite input
    int gram_mode = 0;           // pam_gram_path: 0 tuned, 1 materialized, 2 fused
    bool alive = true;
};

namespace pam {

// Grow buffer `b` of the context to at least `bytes` (synchronizes the stream
// before releasing an older, smaller allocation).
pam_status ensure(pam_ctx *ctx, Buf b, size_t bytes);
template <typename T>
T *wsp(pam_ctx *ctx, Buf b) { return reinterpret_cast<T *>(ctx->ws.ptr[b]); }

__host__ __device__ inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Host-side helpers shared by the API files.
pam_status upload(pam_ctx *ctx, Buf b, const void *host, size_t bytes);
// Copy `bytes` of host data to device address `dst` through the staging buffer.
pam_status upload_to(pam_ctx *ctx, void *dst, const void *host, size_t bytes);

// Padded sizes of the design/Gram workspace for a dictionary capacity.
inline int32_t mpad_of(int32_t m_cap) { return (int32_t)round_up((int64_t)m_cap + 1, 64); }
inline int32_t npad_of(int32_t n_max) { return (int32_t)round_up(n_max > 0 ? n_max : 1, 32); }

// Brackets the launches made during its lifetime with timing events of
// kind `kind` when timing is enabled on the context (kind < 0: no events).
class KernelTimer {
  public:
    KernelTimer(pam_ctx *ctx, int kind);
    ~KernelTimer();
  private:
    pam_ctx *ctx_;
    int kind_;
    hipEvent_t start_ = nullptr;
};

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; every launcher enqueues on ctx->stream and
// returns PAM_OK or PAM_ERR_HIP).
struct FitArgs {
    int32_t n_sub, dim, m_cap, mpad, npad, n_max;
    int32_t sub_begin, sub_count;   // subdomain range of this launch
    const int64_t *off;
    const double *x, *y;
    const int32_t *m;
    const double *c, *sigma;
    double lambda1, lambda2;
    const double *lambda1_sub, *lambda2_sub;
    int32_t precision, cd_sweeps, max_iter, warm_start;
    const uint8_t *hint;
    double *beta;
    pam_fit_stats *stats;
    const int32_t *active;          // [n_sub] 1 = fit this subdomain (refinement), or NULL
    int32_t basis;                  // PAM_BASIS_SHEPARD or PAM_BASIS_PLAIN
    int32_t team;                   // workgroups per subdomain in the solve (1, 2 or 4)
    int32_t team_min;               // active-set size from which a team shares passes
    int32_t team_idle_us;           // a member's wait for a command before it leaves (0: 10 s)
    int32_t gram_fused;             // 1: row sums + fused Gram tiles; 0: assembly + Gram
};

// Non-finite input check of a fit call: for every subdomain, its sample
// points, data values, element extents (h, may be NULL), centers and widths;
// a subdomain with a NaN / infinite value or a width <= 0 gets bit 2 in the
// per-subdomain flags (BUF_FLAGS) and is counted in ctx->sticky[0].
pam_status launch_check_finite(pam_ctx *ctx, const FitArgs &a, const double *h);
pam_status launch_assemble(pam_ctx *ctx, const FitArgs &a);
pam_status launch_gram(pam_ctx *ctx, const FitArgs &a);
// Fused Gram path (FP32 / BF16): row sums, then Gram tiles that compute the
// design in LDS (same bits as the assembly + Gram path).
pam_status launch_rowsum(pam_ctx *ctx, const FitArgs &a);
pam_status launch_gram_fused(pam_ctx *ctx, const FitArgs &a);
pam_status launch_solve(pam_ctx *ctx, const FitArgs &a);
// Dynamic-LDS attribute of the solve instances for a capacity (host only;
// call before a graph capture), and the team control bytes of a launch.
pam_status solve_prepare(int m_cap, int precision);
size_t solve_team_ctl_bytes(int sub_count);
// Graph-safe fills and copies (kernels, not memset / copy nodes).
pam_status launch_fill_u32(pam_ctx *ctx, void *p, uint32_t v, int64_t n_words);
pam_status launch_copy_i32(pam_ctx *ctx, int32_t *dst, const int32_t *src, int64_t n);
pam_status solve_check_capacity(int m_cap, int precision);   // absolute cap of the solve
__host__ __device__ size_t solve_h_elems(int m_cap);
__host__ __device__ size_t solve_scratch_elems(int m_cap, int npad, int precision, int team, bool vg);
// The dictionary capacity is beyond what the solve's per-center vectors can
// hold in LDS: they then live in the subdomain's scratch (one workgroup each).
bool solve_vectors_global(int m_cap, int precision);
// Workgroups per subdomain for a solve launch of sub_count subdomains: the
// largest of requested (0: 4), 2 and 1 whose grid is resident at once.
int solve_team_size(int sub_count, int m_cap, int precision, int requested);

struct RefineArgs {
    int32_t n_sub, dim, m_cap, n_max;
    const int64_t *off;
    const double *x, *y, *h;
    int32_t *m;
    double *c, *sigma;
    int32_t *level;
    double *beta;
    const int32_t *k_top;           // [n_sub] device
    int32_t m_max, space, round, max_rounds;
    double eta, eps_tol;
    int32_t *elem_level;
    int32_t *active;                // [n_sub] in/out: 1 while refining
    int32_t *m0;                    // [n_sub] center count before the first round
    int32_t *rounds;
    double *round_stats;
    pam_fit_stats *stats;
    int32_t basis;
    const int32_t *flags;           // [n_sub] per-subdomain flags of the round's fit
};

pam_status launch_indicator(pam_ctx *ctx, const RefineArgs &a);

// evaluation (k_eval.hip), also used by the Darcy coefficient
pam_status launch_eval(pam_ctx *ctx, int n_fields, const pam_field *fields, const pam_dict *dict,
                       const double *beta, int dtype, const void *xq, int64_t Q, void *out,
                       int space, int64_t *n_outside);
pam_status launch_eval_blend(pam_ctx *ctx, int n_fields, const pam_field *fields,
                             const pam_dict *dict, const double *beta, double blend, int dtype,
                             const void *xq, int64_t Q, void *out, int space, int64_t *n_outside);
// No-alloc evaluation (pam_eval_noalloc): the scratch array's device address
// is looked up once per device (with the device current) by
// eval_scratch_init; launch_eval_noalloc then runs pam_eval's kernels on it.
pam_status eval_scratch_init(int device);
pam_status launch_eval_noalloc(pam_ctx *ctx, int n_fields, const pam_field *fields,
                               const pam_dict *dict, const double *beta, int dtype, const void *xq,
                               int64_t Q, void *out, int space, int64_t *n_outside);
pam_status launch_mark_enrich(pam_ctx *ctx, const RefineArgs &a);
// PAM_ERR_CAPACITY when the marking cannot rank n_max samples per subdomain.
pam_status mark_check_capacity(int n_max);
// HBM workspace of the marking for subdomains beyond the LDS sort (0 within).
size_t mark_ws_bytes(int n_sub, int n_max);

}  // namespace pam
