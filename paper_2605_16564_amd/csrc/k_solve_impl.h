// Elastic-net solve for every subdomain (gfx950): the unique minimizer of
//   1/2 ||y - W beta||^2 + lambda1 ||beta||_1 + lambda2/2 ||beta||^2
// (Eq. elastic) from the normal products G = W'W, b = W'y (Sec. 3.3: the
// problem is convex and coordinate descent reaches its minimizer).
//
// One block (four waves) per subdomain:
//  1. cyclic coordinate descent sweeps in creation order (warm-up);
//  2. exact sign-consistent active-set iteration (feature-sign search):
//     solve (G_SS + lambda2 I) beta_S = b_S - lambda1 theta_S on the signed
//     active set, discrete line search over the zero crossings, activation of
//     the worst KKT violators; the inverse H of the active block is kept in
//     HBM/L2 and updated by (blocked) bordering when coordinates enter and by
//     a Schur downdate when they leave;
//  3. residual refinement of the reduced system and a KKT certificate in FP64.
// All vectors of the iteration live in LDS; only H and the Gram rows stream
// from memory, in coalesced row order.
#pragma once
#include <float.h>

#include "pam_internal.h"

#include <algorithm>

#ifdef PAM_PHASE_PROFILE
#include <stdio.h>
// per-subdomain phase record of the profile build: [0, 8) microseconds per
// phase, [8, 16) bytes per phase, [16, 28) counts (written by thread 0 at the
// end of the solve, read and printed by the host after each launch)
static constexpr int kPhaseW = 56, kPhaseSubs = 8192;
static __device__ double g_phase[kPhaseSubs * kPhaseW];
#define PHASE_MARK(k) do { if (threadIdx.x == 0) { long long _t = wall_clock64(); ph[k] += _t - ph_last; ph_last = _t; phb[k] += v.bytes - phb_last; phb_last = v.bytes; } } while (0)
// sub-phases (thread 0's clock at the block's sync points): SUB_START opens a
// region, SUB(k) adds the time since the last mark to slot k
#define SUB_START() do { if (threadIdx.x == 0) v.sp[23] = wall_clock64(); } while (0)
#define SUB(k) do { if (threadIdx.x == 0) { long long _t = wall_clock64(); v.sp[k] += _t - v.sp[23]; v.sp[23] = _t; } } while (0)
#else
#define PHASE_MARK(k) do { } while (0)
#define SUB_START() do { } while (0)
#define SUB(k) do { } while (0)
#endif

namespace pam {

static constexpr int kT = 512;
static constexpr int kW = kT / 64;
static constexpr int kB = 8;       // coordinates activated per blocked bordering step
static constexpr int kAdd = 16;    // violators activated per consistent iteration
static constexpr int kInit = 24;   // coordinates per activation call when a block is built from scratch
static constexpr int kR = 1;       // GEMV outputs per thread per pass
static constexpr int kTile = 128;  // rows staged in LDS per bordering tile
static constexpr int kFz = 8;      // coordinates frozen before one batched downdate
static constexpr int kQ = 24;      // rows of the low-rank update scratch (>= kFz + 2 kB)
static constexpr int kPass = kR * kT;
static constexpr int kUR = 16;     // rows of H in flight per thread in the bordering product
static constexpr int kHR = 8;      // rows of H per batch in the low-rank updates (two batches in flight)
static constexpr int kPolishMax = 30;  // FP64 conjugate-gradient steps of the polish
static constexpr int kIncMax = 384;    // incremental solution updates between full solves
// a sign-consistent carried solution is confirmed by a full solve only when
// more than kConfirm incremental updates separate it from the last full solve
// (each loses about eps cond(G); the steps it accepts are still certified by
// the reduced-system residual and the KKT check at the end)
static constexpr int kConfirm = 192;
static_assert(kFz <= kB && kFz + 2 * kB <= kQ && kInit <= kQ, "deferred blocks fit the update scratch");

// A team of up to kTeamMax workgroups may serve one subdomain (the launch is
// sized so that the device holds all of its workgroups at once, by the
// occupancy query; residency is needed for speed only, never for progress,
// since every wait below is bounded): its first workgroup (the leader) runs the whole
// iteration; once the active set reaches team_min coordinates, every pass
// that streams the active-block inverse H or the Gram is split into row
// slices, one per member (the leader's included), and the leader sums the
// members' partial results in member order. Commands and completions go
// through a per-team control block (one 128-byte line each) with agent-scope
// release/acquire. Every wait is bounded: a member idle for longer than its
// bound leaves, and the leader does its rows from then on; a member that
// neither answers nor leaves within kTeamWait leaves the leader alone, and
// that subdomain's result is reported NOCONV.
static constexpr int kTeamMax = 4;
static constexpr int kCtl = 16 * (kTeamMax + 1);       // u64 control words per team
static constexpr long long kTeamWait = 1000000000LL;   // 10 s of the 100 MHz constant clock
static constexpr unsigned kWaitVm0 = 0x0F70;           // s_waitcnt vmcnt(0) (gfx9 encoding)
enum TeamOp { OP_QUIT = 0, OP_GEMV = 1, OP_UPASS = 2, OP_UPDATE = 3, OP_GRAD = 4 };

// (force-inlined bodies: a call from the kernel would make it a non-leaf
// function with the calling convention's register cost)
__host__ __device__ __forceinline__ size_t ldh_of(int m_cap) { return (size_t)round_up(m_cap, kPass); }
__host__ __device__ __forceinline__ size_t h_elems_of(int m_cap) { return (size_t)(m_cap + 1) * ldh_of(m_cap); }
// The iteration's per-center vectors (57 B per center: six FP64 vectors, two
// int vectors, one sign byte) in FP64 slots: 7 Mc + Mc / 8, Mc = m_cap rounded
// up to 8.
__host__ __device__ __forceinline__ size_t vec_elems_of(int m_cap) {
    const size_t mc = (size_t)round_up(m_cap, 8);
    return 7 * mc + mc / 8 + 8;
}
__host__ __device__ __forceinline__ size_t scratch_elems_of(int m_cap, int npad, int precision, int team,
                                                             bool vg = false) {
    // blocked-bordering rows [3][kQ][m_cap], then for the FP64 phase of the
    // low-precision modes: -1/(2 sigma^2) [m_cap], three CG vectors [3][m_cap],
    // two per-sample vectors [2][npad] and the FP64 design W64 [m_cap][npad];
    // with a team: partial results [kTeamMax][kB][m_cap], the input vector,
    // beta by coordinate and the active list [3][m_cap]; with vg (the
    // dictionary is too large for the vectors to sit in LDS) the iteration's
    // vectors last
    const size_t w64 = precision == PAM_PREC_F64 ? 0 : (size_t)m_cap * npad;
    const size_t tm = team > 1 ? (size_t)(kTeamMax * kB + 3) * m_cap : 0;
    return (size_t)3 * kQ * m_cap + (size_t)4 * m_cap + (size_t)2 * npad + w64 + tm + (vg ? vec_elems_of(m_cap) : 0);
}

// ---------------------------------------------------------------- reductions
struct Red {
    double v[kW * 16];
    int i[kW];
    int flag;
    int count;
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double bsum(double v, Red &r) {
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) r.v[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kW; ++w) t += r.v[w];
    __syncthreads();
    return t;
}

template <int K>
__device__ __forceinline__ void bsum_vec(double (&v)[K], Red &r) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = wsum(v[k]);
        if ((threadIdx.x & 63) == 0) r.v[(threadIdx.x >> 6) * K + k] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kW; ++w) t += r.v[w * K + k];
        v[k] = t;
    }
    __syncthreads();
}

struct VI { double v; int i; };
__device__ __forceinline__ VI vmax(VI a, VI b) {
    if (b.i < 0) return a;
    if (a.i < 0) return b;
    if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
    return a;
}
__device__ __forceinline__ VI bargmax(VI x, Red &r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        VI y;
        y.v = __shfl_xor(x.v, o, 64);
        y.i = __shfl_xor(x.i, o, 64);
        x = vmax(x, y);
    }
    if ((threadIdx.x & 63) == 0) { r.v[threadIdx.x >> 6] = x.v; r.i[threadIdx.x >> 6] = x.i; }
    __syncthreads();
    VI t; t.v = -1.0; t.i = -1;
#pragma unroll
    for (int w = 0; w < kW; ++w) { VI y; y.v = r.v[w]; y.i = r.i[w]; t = vmax(t, y); }
    __syncthreads();
    return t;
}
__device__ __forceinline__ double bmax(double v, Red &r) {
    VI x; x.v = v; x.i = threadIdx.x;
    return bargmax(x, r).v;
}
// AND over the block of a per-thread predicate.
__device__ __forceinline__ bool ball(bool p, Red &r) {
    if (threadIdx.x == 0) r.flag = 1;
    __syncthreads();
    if (!p) r.flag = 0;
    __syncthreads();
    const bool res = r.flag != 0;
    __syncthreads();
    return res;
}

__device__ __forceinline__ double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

// ---------------------------------------------------------------- state
template <typename TG>
struct Sv {
    const TG *G;           // Gram [mpad][mpad]; column M holds b
    int mpad, M, m_cap;
    size_t ldh;
    double l1, l2;
    double *H;             // [m_cap+1][ldh] inverse of the active block
    double *Ag, *U, *V;    // [kB][m_cap] scratch for blocked bordering
    double *g, *beta;      // LDS, by coordinate
    double *b;             // LDS, by coordinate: b = W'y (column M of the Gram)
    double *z, *rhs, *u;   // LDS, by active position
    int *S, *pos;          // LDS
    signed char *th;       // LDS
    int s;                 // active-set size (uniform)
    double bytes;          // algorithmic bytes streamed (Gram rows, H)
    int r;                 // frozen positions awaiting the batched downdate
    int pend;              // rank of a deferred update (rows [0, pend) of U, V)
    int fz;                // frozen positions whose downdate is part of the deferred update
    int *Rp;               // LDS [kFz] frozen positions
    double *Cri;           // LDS [kFz*kFz] inverse of H[R, R]
    // team (T > 1): see kTeamMax. The team scratch holds partial results
    // [kTeamMax][kB * m_cap], the input vector [m_cap], beta by coordinate
    // [m_cap] and the active list [m_cap]; T drops to 1 when a member did
    // not answer in time (tsh[3] then records the failure).
    int T, team_min;
    long long idle;            // constant-clock ticks a member waits for a command before leaving
    unsigned long long *ctl;   // [kCtl] command, arguments, completion words
    double *part;              // team scratch
    unsigned *tsh;             // LDS [5]: command broadcast, commands posted, failure
#ifdef PAM_PHASE_PROFILE
    long long *sp;             // LDS [24] sub-phase clocks
#endif
    __device__ double *xin() const { return part + (size_t)kTeamMax * kB * m_cap; }
    __device__ double *bco() const { return part + (size_t)(kTeamMax * kB + 1) * m_cap; }
    __device__ int *Sg() const { return reinterpret_cast<int *>(part + (size_t)(kTeamMax * kB + 2) * m_cap); }
};

template <typename TG>
__device__ __forceinline__ bool team_on(const Sv<TG> &v) { return v.T > 1 && v.s >= v.team_min; }

// rows [row0(k), row0(k+1)) of an s-row pass belong to member k
__device__ __forceinline__ int team_row0(int k, int s, int T) { return (int)((long long)k * s / T); }

__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Leader: publish a command (every wave's earlier stores are in L2 before
// the barrier; the release store writes them back for the other members).
template <typename TG>
__device__ __forceinline__ void team_post(Sv<TG> &v, int op, int s, int n) {
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned seq = ++v.tsh[4];
        v.ctl[1] = (unsigned long long)op;
        v.ctl[2] = (unsigned long long)s;
        v.ctl[3] = (unsigned long long)n;
        __hip_atomic_store(&v.ctl[0], (unsigned long long)seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// A member whose wait for a command ran past its idle bound leaves and marks
// its completion word kGone; it never started the pending command, if any.
static constexpr unsigned long long kGone = ~0ull;

template <typename TG>
__device__ __forceinline__ void team_slice(Sv<TG> &v, int op, int s, int n, int k, double *tile);

// Leader: wait for every member's completion of the last command (bounded).
// The slices of members that have left are done here; a member that neither
// completes nor leaves in time leaves the leader alone for the rest of the
// solve (the result is then reported as not certified).
template <typename TG>
__device__ __forceinline__ void team_join(Sv<TG> &v, int op, int s, int n, double *tile) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long seq = v.tsh[4];
        const long long t0 = wall_clock64();
        bool ok = true;
        unsigned gone = 0;
        for (int k = 1; k < v.T && ok; ++k) {
            unsigned long long d;
            while ((d = ld_relaxed(&v.ctl[16 * k])) != seq && d != kGone) {
                if (wall_clock64() - t0 > kTeamWait) { ok = false; break; }
                __builtin_amdgcn_s_sleep(2);
            }
            if (d == kGone) gone |= 1u << k;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!ok) v.tsh[3] = 1;
        v.tsh[0] = gone;
    }
    __syncthreads();
    const unsigned gone = v.tsh[0];
    if (v.tsh[3]) {
        v.T = 1;   // uniform: the leader goes on alone
        return;
    }
    for (int k = 1; k < v.T; ++k)
        if (gone & (1u << k)) team_slice(v, op, s, n, k, tile);
}

template <typename TG>
__device__ __forceinline__ double Gat(const Sv<TG> &v, int i, int j) {
    return (double)v.G[(size_t)i * v.mpad + j];
}

// out_i = sum_{r0 <= j < r1} H[j][i] in_j, i < s (H symmetric; rows
// streamed coalesced, eight rows in flight per thread).
template <int R, typename TG>
__device__ __forceinline__ void hgemv_r(Sv<TG> &v, const double *in, double *out, int r0, int r1) {
    constexpr int kRows = 8;   // rows loaded before use
    const int s = v.s;
    for (int base = 0; base < s; base += R * kT) {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        const double *Hc = v.H + base + threadIdx.x;
        int jj = r0;
        for (; jj + kRows <= r1; jj += kRows) {
            double h[kRows][R];
#pragma unroll
            for (int q = 0; q < kRows; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) h[q][r] = Hc[(size_t)(jj + q) * v.ldh + r * kT];
#pragma unroll
            for (int q = 0; q < kRows; ++q) {
                const double x = in[jj + q];
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += h[q][r] * x;
            }
        }
        for (; jj < r1; ++jj) {
            const double x = in[jj];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += Hc[(size_t)jj * v.ldh + r * kT] * x;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + threadIdx.x + r * kT;
            if (i < s) out[i] = acc[r];
        }
    }
    __syncthreads();
}

// rows [r0, r1) of out = H in, up to four outputs per thread so that more
// rows are in flight
template <typename TG>
__device__ __forceinline__ void hgemv_rows(Sv<TG> &v, const double *in, double *out, int r0, int r1) {
    if (v.s <= kT) hgemv_r<1>(v, in, out, r0, r1);
    else if (v.s <= 2 * kT) hgemv_r<2>(v, in, out, r0, r1);
    else hgemv_r<4>(v, in, out, r0, r1);
}

// out_i = sum_j H[j][i] in_j, i < s; a team sums its members' row slices
// (in member order).
template <typename TG>
__device__ __forceinline__ void hgemv(Sv<TG> &v, const double *in, double *out) {
    const int s = v.s;
    v.bytes += 8.0 * (double)s * (double)s;
    if (!team_on(v)) {
        SUB_START();
        hgemv_rows(v, in, out, 0, s);
        SUB(14);
        return;
    }
    double *xin = v.xin();
    for (int i = threadIdx.x; i < s; i += kT) xin[i] = in[i];
    team_post(v, OP_GEMV, s, 0);
    team_slice(v, OP_GEMV, s, 0, 0, nullptr);
    team_join(v, OP_GEMV, s, 0, nullptr);
    const size_t lp = (size_t)kB * v.m_cap;
    for (int i = threadIdx.x; i < s; i += kT) {
        double acc = v.part[i];
        for (int k = 1; k < v.T; ++k) acc += v.part[k * lp + i];
        out[i] = acc;
    }
    __syncthreads();
}

// H[i][j] += sum_q Vr[q][i] Ur[q][j] for r0 <= i < r1, j < s and q < nq
// (nq <= NQ): thread-owned columns j keep Ur[.][j] in registers, rows i
// stream in batches of eight with Vr[.][i] staged in LDS tiles.
template <int NQ, typename TG>
__device__ __forceinline__ void hupdate(Sv<TG> &v, int s, int nq, const double *Vr, const double *Ur, double *tile,
                                        int r0, int r1) {
    for (int jb = 0; jb < s; jb += kT) {
        const int j = jb + threadIdx.x;
        const bool live = j < s;
        double uj[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) uj[q] = (live && q < nq) ? Ur[(size_t)q * v.m_cap + j] : 0.0;
        double *Hc = v.H + j;
        for (int t0 = r0; t0 < r1; t0 += kTile) {
            const int tn = min(kTile, r1 - t0);
            __syncthreads();
            for (int e = threadIdx.x; e < NQ * kTile; e += kT) {
                const int q = e / kTile, r = e - q * kTile;
                tile[e] = (q < nq && r < tn) ? Vr[(size_t)q * v.m_cap + t0 + r] : 0.0;
            }
            __syncthreads();
            if (!live) continue;
            // batches of kHR rows, the next batch's loads issued before this
            // batch's stores (rows are disjoint), so that loads stay in
            // flight while the stores drain
            const int nfull = tn / kHR;
            int r = 0;
            if (nfull > 0) {
                double hv[kHR];
#pragma unroll
                for (int e = 0; e < kHR; ++e) hv[e] = Hc[(size_t)(t0 + e) * v.ldh];
                for (int bi = 0; bi < nfull; ++bi, r += kHR) {
                    const bool more = bi + 1 < nfull;
                    double hn[kHR];
                    if (more) {
#pragma unroll
                        for (int e = 0; e < kHR; ++e) hn[e] = Hc[(size_t)(t0 + r + kHR + e) * v.ldh];
                    }
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const double uq = uj[q];
#pragma unroll
                        for (int e = 0; e < kHR; ++e) hv[e] += tile[q * kTile + r + e] * uq;
                    }
                    double *h = Hc + (size_t)(t0 + r) * v.ldh;
#pragma unroll
                    for (int e = 0; e < kHR; ++e) h[(size_t)e * v.ldh] = hv[e];
                    if (more) {
#pragma unroll
                        for (int e = 0; e < kHR; ++e) hv[e] = hn[e];
                    }
                }
            }
            for (; r < tn; ++r) {
                double *h = Hc + (size_t)(t0 + r) * v.ldh;
                double h0 = h[0];
#pragma unroll
                for (int q = 0; q < NQ; ++q) h0 += tile[q * kTile + r] * uj[q];
                h[0] = h0;
            }
        }
    }
    __syncthreads();
}

// H += V' U over all s rows (nq <= kB rank): shared by the team in row
// slices once the block is large.
template <typename TG>
__device__ __forceinline__ void hupdate_rows(Sv<TG> &v, int s, int nq, double *tile, int r0, int r1) {
    if (nq <= kB) hupdate<kB>(v, s, nq, v.V, v.U, tile, r0, r1);
    else if (nq <= 2 * kB) hupdate<2 * kB>(v, s, nq, v.V, v.U, tile, r0, r1);
    else hupdate<kQ>(v, s, nq, v.V, v.U, tile, r0, r1);
}

template <typename TG>
__device__ __forceinline__ void hupdate_all(Sv<TG> &v, int s, int nq, double *tile) {
    if (v.T > 1 && s >= v.team_min) {
        team_post(v, OP_UPDATE, s, nq);
        team_slice(v, OP_UPDATE, s, nq, 0, tile);
        team_join(v, OP_UPDATE, s, nq, tile);
    } else {
        hupdate_rows(v, s, nq, tile, 0, s);
    }
}

// out[q][i] = sum_{r0 <= t < r1} H[t][i] Ag[q][t] for i < s, q < nb (rows
// [q * m_cap, ...) of out): one pass over rows [r0, r1) of H for all nb
// columns, the rows of Ag staged through LDS tiles.
template <int NB, typename TG>
__device__ __forceinline__ void upass_n(Sv<TG> &v, int nb, int r0, int r1, double *out, double *tile);

template <typename TG>
__device__ __forceinline__ void upass(Sv<TG> &v, int nb, int r0, int r1, double *out, double *tile) {
    upass_n<kB>(v, nb, r0, r1, out, tile);
}

// upass for up to NB columns (rows [0, nb) of Ag): NB = 2 kB serves two
// consecutive bordering blocks in one pass over H.
template <int NB, typename TG>
__device__ __forceinline__ void upass_n(Sv<TG> &v, int nb, int r0, int r1, double *out, double *tile) {
    const int s = v.s;
    for (int base = 0; base < s; base += kPass) {
        double acc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = 0.0;
        const double *Hc = v.H + base + threadIdx.x;
        for (int t0 = r0; t0 < r1; t0 += kTile) {
            const int tn = min(kTile, r1 - t0);
            __syncthreads();
            for (int e = threadIdx.x; e < NB * kTile; e += kT) {
                const int q = e / kTile, r = e - q * kTile;
                tile[e] = (q < nb && r < tn) ? v.Ag[(size_t)q * v.m_cap + t0 + r] : 0.0;
            }
            __syncthreads();
            int r = 0;
            for (; r + kUR <= tn; r += kUR) {
                double h[kUR];
#pragma unroll
                for (int e = 0; e < kUR; ++e) h[e] = Hc[(size_t)(t0 + r + e) * v.ldh];
#pragma unroll
                for (int e = 0; e < kUR; ++e)
#pragma unroll
                    for (int q = 0; q < NB; ++q) acc[q] += h[e] * tile[q * kTile + r + e];
            }
            for (; r < tn; ++r) {
                const double h0 = Hc[(size_t)(t0 + r) * v.ldh];
#pragma unroll
                for (int q = 0; q < NB; ++q) acc[q] += h0 * tile[q * kTile + r];
            }
        }
        const int i = base + threadIdx.x;
        if (i < s)
            for (int q = 0; q < nb; ++q) out[(size_t)q * v.m_cap + i] = acc[q];
    }
    __syncthreads();
}

template <typename TG>
__device__ __forceinline__ void drop_frozen(Sv<TG> &v);

// sum_i x[i] y[i] over i = l16, l16 + 16, ... < s (one lane of a 16-lane
// group): four partial sums, so that eight loads are in flight per lane
__device__ __forceinline__ double dot16(const double *x, const double *y, int l16, int s) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = l16;
    for (; i + 48 < s; i += 64) {
        const double x0 = x[i], x1 = x[i + 16], x2 = x[i + 32], x3 = x[i + 48];
        const double y0 = y[i], y1 = y[i + 16], y2 = y[i + 32], y3 = y[i + 48];
        a0 += x0 * y0;
        a1 += x1 * y1;
        a2 += x2 * y2;
        a3 += x3 * y3;
    }
    for (; i < s; i += 16) a0 += x[i] * y[i];
    return (a0 + a1) + (a2 + a3);
}

// Blocked bordering: append the nb (<= kB) coordinates ks[] to the active
// set. With A_SB = G[S, B], U = H A_SB, C = A_BB + lambda2 I - A_SB' U,
//   H <- [[H + U C^-1 U', -U C^-1], [-C^-1 U', C^-1]].
// Returns false (set unchanged) if C is not numerically positive definite.
// Rows of A_SB and of V = U C^-1 are staged through LDS in tiles so that
// the streaming passes over H read them as broadcasts.
// With upd_z, v.z holds H r_S for the current block (r = b - lambda1 theta)
// on entry and the solution for the enlarged block on return:
//   z_S <- z_S + V (U' r_S - r_B),  z_B = C^-1 (r_B - U' r_S).
// With defer (and nothing pending), the update of the old block is left
// pending: the border rows are written, V and U stay in rows [0, nb) of the
// scratch (zero on the new positions) and v.pend = nb. The next block then
// reads the stored H, corrects its U by the pending rank (U += Vp (Up' A))
// and applies both updates in one rank-(pend + nb) pass, so a pair of blocks
// streams H three times instead of four.
template <typename TG>
__device__ __forceinline__ bool add_block(Sv<TG> &v, const int *ks, int nb, Red &red, double *cinv, double *tile,
                                          bool upd_z = false, bool defer = false, const int *ks_next = nullptr,
                                          int nb_next = 0, bool pre = false) {
    const int s = v.s, pend = v.pend;
    double *Ub = v.U + (size_t)pend * v.m_cap, *Vb = v.V + (size_t)pend * v.m_cap;
    v.bytes += (pre ? 0.0 : 8.0 * (double)s * (double)s) + (double)(nb + nb_next) * s * sizeof(TG);
    SUB_START();
    // A_SB: the nb Gram rows of the block at the active coordinates (all
    // loads of a thread issued before its stores); with nb_next, the next
    // block's rows too (rows [kB, kB + nb_next) of Ag), for a shared pass
    for (int i = threadIdx.x; i < s; i += kT) {
        const int k = v.S[i];
        TG gq[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) gq[q] = q < nb ? v.G[(size_t)ks[q] * v.mpad + k] : (TG)0;
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (q < nb) v.Ag[(size_t)q * v.m_cap + i] = (double)gq[q];
        if (nb_next > 0) {
#pragma unroll
            for (int q = 0; q < kB; ++q) gq[q] = q < nb_next ? v.G[(size_t)ks_next[q] * v.mpad + k] : (TG)0;
#pragma unroll
            for (int q = 0; q < kB; ++q)
                if (q < nb_next) v.Ag[(size_t)(kB + q) * v.m_cap + i] = (double)gq[q];
        }
    }
    __syncthreads();
    SUB(0);
    if (pre) {
        // U over the old positions i < k0 came from the previous block's
        // shared pass (H of the block before it, which that block left
        // unchanged: it deferred its update); add the previous block's border
        // rows k0.. of H (in the order the pass over H would), and take the
        // new positions' entries as dots of their border rows with A_SB
        const int k0 = s - kB;
        for (int i = threadIdx.x; i < k0; i += kT) {
            double hb[kB];
#pragma unroll
            for (int p = 0; p < kB; ++p) hb[p] = v.H[(size_t)(k0 + p) * v.ldh + i];
            for (int q = 0; q < nb; ++q) {
                double acc = Ub[(size_t)q * v.m_cap + i];
#pragma unroll
                for (int p = 0; p < kB; ++p) acc += hb[p] * v.Ag[(size_t)q * v.m_cap + k0 + p];
                Ub[(size_t)q * v.m_cap + i] = acc;
            }
        }
        for (int pair0 = 0; pair0 < kB * kB; pair0 += kT / 16) {
            const int pair = pair0 + (threadIdx.x >> 4), l16 = threadIdx.x & 15;
            const int p = pair / kB, q = pair % kB;
            double acc = 0.0;
            if (pair < kB * kB && q < nb)
                acc = dot16(v.H + (size_t)(k0 + p) * v.ldh, v.Ag + (size_t)q * v.m_cap, l16, s);
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
            if (l16 == 0 && pair < kB * kB && q < nb) Ub[(size_t)q * v.m_cap + k0 + p] = acc;
        }
        __syncthreads();
    } else if (nb_next > 0) {
        // one pass over H for this block's nb = kB columns and the next
        // block's nb_next: rows [0, kB + nb_next) of Ub (the next block's
        // rows start where its own Ub will, this block deferring its update)
        upass_n<2 * kB>(v, kB + nb_next, 0, s, Ub, tile);
    } else if (!team_on(v)) {
        // U = H A_SB: one pass over H for all nb columns
        upass(v, nb, 0, s, Ub, tile);
    } else {
        team_post(v, OP_UPASS, s, nb);
        team_slice(v, OP_UPASS, s, nb, 0, tile);
        team_join(v, OP_UPASS, s, nb, tile);
        const size_t lp = (size_t)kB * v.m_cap;
        for (int e = threadIdx.x; e < nb * s; e += kT) {
            const int q = e / s, i = e - q * s;
            const size_t o = (size_t)q * v.m_cap + i;
            double acc = v.part[o];
            for (int k = 1; k < v.T; ++k) acc += v.part[k * lp + o];
            Ub[o] = acc;
        }
        __syncthreads();
    }
    SUB(1);
    if (pend > 0) {
        // the stored block lacks the pending V_p U_p' on the old positions:
        // U += V_p (U_p' A_SB), with X = U_p' A_SB (pend x nb) in tile[kB*kB ...)
        constexpr int kPairs = (kQ - kB) * kB;
        double *X = tile + kB * kB;
        for (int pair0 = 0; pair0 < kPairs; pair0 += kT / 16) {
            const int pair = pair0 + (threadIdx.x >> 4), l16 = threadIdx.x & 15;
            const int p = pair / kB, q = pair % kB;
            double acc = 0.0;
            if (pair < kPairs && p < pend && q < nb)
                acc = dot16(v.U + (size_t)p * v.m_cap, v.Ag + (size_t)q * v.m_cap, l16, s);
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
            if (l16 == 0 && pair < kPairs) X[pair] = acc;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < s; i += kT) {
            double acc[kB];
#pragma unroll
            for (int q = 0; q < kB; ++q) acc[q] = q < nb ? Ub[(size_t)q * v.m_cap + i] : 0.0;
            for (int p = 0; p < pend; ++p) {
                const double vp = v.V[(size_t)p * v.m_cap + i];
#pragma unroll
                for (int q = 0; q < kB; ++q) acc[q] += vp * X[p * kB + q];
            }
#pragma unroll
            for (int q = 0; q < kB; ++q)
                if (q < nb) Ub[(size_t)q * v.m_cap + i] = acc[q];
        }
        __syncthreads();
    }
    SUB(2);
    // C = A_BB + lambda2 I - A_SB' U: 16 threads per (p, q) pair
    for (int pair0 = 0; pair0 < kB * kB; pair0 += kT / 16) {
        const int pair = pair0 + (threadIdx.x >> 4), l16 = threadIdx.x & 15;
        const int p = pair / kB, q = pair % kB;
        double acc = 0.0;
        if (pair < kB * kB && p < nb && q < nb)
            acc = dot16(v.Ag + (size_t)p * v.m_cap, Ub + (size_t)q * v.m_cap, l16, s);
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
        if (l16 == 0 && pair < kB * kB) tile[pair] = acc;
    }
    // A_BB + lambda2 I in LDS for the factorization below (after X)
    double *Abb = tile + kB * kB + (kQ - kB) * kB;
    if ((int)threadIdx.x < nb * nb) {
        const int p = threadIdx.x / nb, q = threadIdx.x - (threadIdx.x / nb) * nb;
        Abb[p * kB + q] = Gat(v, ks[p], ks[q]) + (p == q ? v.l2 : 0.0);
    }
    __syncthreads();
    SUB(3);
    if (threadIdx.x < 64) {
        // C^-1 by Gauss-Jordan elimination in wave 0, one lane per entry of
        // the (padded) kB x kB block; C is symmetric positive definite, so the
        // pivots are the Schur complements that a Cholesky factorization would
        // take roots of, checked against the same threshold
        static_assert(kB * kB == 64, "one lane per entry of the bordering block");
        const int lane = threadIdx.x, i = lane / kB, j = lane % kB;
        double e = (i < nb && j < nb) ? Abb[i * kB + j] - tile[i * kB + j] : (i == j ? 1.0 : 0.0);
        int ok = 1;
        for (int k = 0; k < nb; ++k) {
            const double akk = __shfl(e, k * kB + k, 64);
            const double aik = __shfl(e, i * kB + k, 64);
            const double akj = __shfl(e, k * kB + j, 64);
            if (!(akk > 1e-14 * Abb[k * kB + k])) { ok = 0; break; }   // uniform over the wave
            const double ip = 1.0 / akk;
            if (i == k && j == k) e = ip;
            else if (i == k) e = akj * ip;
            else if (j == k) e = -aik * ip;
            else e = e - aik * akj * ip;
        }
        const double et = __shfl(e, j * kB + i, 64);
        if (ok && i < nb && j < nb) cinv[i * kB + j] = 0.5 * (e + et);
        if (lane == 0) red.flag = ok;
    }
    __syncthreads();
    const bool ok = red.flag != 0;
    __syncthreads();
    SUB(4);
    if (!ok) return false;
    // V = U C^-1
    for (int i = threadIdx.x; i < s; i += kT) {
        double uu[kB];
#pragma unroll
        for (int p = 0; p < kB; ++p) uu[p] = p < nb ? Ub[(size_t)p * v.m_cap + i] : 0.0;
        for (int q = 0; q < nb; ++q) {
            double val = 0.0;
#pragma unroll
            for (int p = 0; p < kB; ++p) val += uu[p] * (p < nb ? cinv[p * kB + q] : 0.0);
            Vb[(size_t)q * v.m_cap + i] = val;
        }
    }
    __syncthreads();
    SUB(5);
    if (upd_z) {
        double ur[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) ur[q] = 0.0;
        for (int i = threadIdx.x; i < s; i += kT) {
            const int k = v.S[i];
            const double ri = v.b[k] - v.l1 * (double)v.th[k];
#pragma unroll
            for (int q = 0; q < kB; ++q) ur[q] += q < nb ? Ub[(size_t)q * v.m_cap + i] * ri : 0.0;
        }
        bsum_vec<kB>(ur, red);
        double w[kB];   // U' r_S - r_B
#pragma unroll
        for (int q = 0; q < kB; ++q)
            w[q] = q < nb ? ur[q] - (v.b[ks[q]] - v.l1 * (double)v.th[ks[q]]) : 0.0;
        for (int i = threadIdx.x; i < s; i += kT) {
            double acc = v.z[i];
#pragma unroll
            for (int q = 0; q < kB; ++q) acc += q < nb ? Vb[(size_t)q * v.m_cap + i] * w[q] : 0.0;
            v.z[i] = acc;
        }
        if ((int)threadIdx.x < nb) {
            double acc = 0.0;
            for (int q = 0; q < nb; ++q) acc -= cinv[threadIdx.x * kB + q] * w[q];
            v.z[s + threadIdx.x] = acc;
        }
        __syncthreads();
    }
    // H[i][j] += sum_q V[q][i] U[q][j] over the old block (with the pending
    // rows, which are zero on the pending block's own positions)
    // defer when the next block still fits the scratch rows
    const bool keep = defer && pend + nb + kB <= kQ;
    SUB(6);
    if (!keep) {
        v.bytes += 16.0 * (double)s * (double)s;
        hupdate_all(v, s, pend + nb, tile);
    }
    SUB(7);
    for (int j = threadIdx.x; j < s; j += kT)
        for (int q = 0; q < nb; ++q) {
            const double val = -Vb[(size_t)q * v.m_cap + j];
            v.H[(size_t)(s + q) * v.ldh + j] = val;
            v.H[(size_t)j * v.ldh + s + q] = val;
        }
    if (threadIdx.x < nb * nb) {
        const int p = threadIdx.x / nb, q = threadIdx.x % nb;
        v.H[(size_t)(s + p) * v.ldh + s + q] = cinv[p * kB + q];
    }
    if (threadIdx.x < nb) {
        v.S[s + threadIdx.x] = ks[threadIdx.x];
        v.pos[ks[threadIdx.x]] = s + threadIdx.x;
    }
    if (keep) {
        // the pending factors (earlier ones and this block's) vanish on the
        // new positions
        for (int e = threadIdx.x; e < (pend + nb) * nb; e += kT) {
            const int q = e / nb, i = s + e % nb;
            v.U[(size_t)q * v.m_cap + i] = 0.0;
            v.V[(size_t)q * v.m_cap + i] = 0.0;
        }
    }
    __syncthreads();
    SUB(8);
    v.pend = keep ? pend + nb : 0;
    v.s = s + nb;
    if (!keep && v.fz > 0) drop_frozen(v);
    return true;
}

// Apply a deferred bordering update (rank v.pend) to the stored block.
template <typename TG>
__device__ __forceinline__ void flush_pending(Sv<TG> &v, double *tile) {
    if (v.pend == 0) return;
    v.bytes += 16.0 * (double)v.s * (double)v.s;
    SUB_START();
    hupdate_all(v, v.s, v.pend, tile);
    SUB(7);
    v.pend = 0;
    if (v.fz > 0) drop_frozen(v);
}

// Drop active position p (no update of H): the last position moves into p.
template <typename TG>
__device__ __forceinline__ void drop_position(Sv<TG> &v, int p) {
    const int last = v.s - 1;
    const int kp = v.S[p];
    if (p != last) {
        for (int j = threadIdx.x; j < last; j += kT) {
            if (j == p) continue;
            const double val = v.H[(size_t)last * v.ldh + j];
            v.H[(size_t)p * v.ldh + j] = val;
            v.H[(size_t)j * v.ldh + p] = val;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            v.H[(size_t)p * v.ldh + p] = v.H[(size_t)last * v.ldh + last];
            const int kl = v.S[last];
            v.S[p] = kl;
            v.pos[kl] = p;
            v.z[p] = v.z[last];   // the maintained solution follows its position
        }
    }
    if (threadIdx.x == 0) v.pos[kp] = -1;
    __syncthreads();
    v.s = last;
}

// Freeze active position p: its coordinate is held at zero without touching
// H. With W = H[:, R] (rows of H, by symmetry) and C = H[R, R], the inverse of
// the remaining block is H - W C^-1 W'; C^-1 grows by bordering.
//
// With upd_z, v.z holds the solution on the current live positions and is
// carried to the block without p: z <- z - h z_p / h_pp, h the column p of
// the effective inverse H - W C^-1 W' (before p joins the frozen set).
template <typename TG>
__device__ __forceinline__ void freeze(Sv<TG> &v, int p, bool upd_z = false) {
    const int s = v.s, r = v.r;
    v.bytes += 8.0 * s;
    SUB_START();
    for (int i = threadIdx.x; i < s; i += kT) v.U[(size_t)r * v.m_cap + i] = v.H[(size_t)p * v.ldh + i];
    __syncthreads();
    // H[R, p] and H[p, p] into LDS in parallel for the serial part below
    if ((int)threadIdx.x <= r) {
        double *c = v.Cri + kFz * kFz;
        c[threadIdx.x] = v.U[(size_t)threadIdx.x * v.m_cap + p];   // row r holds H[p, .]
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *c = v.Cri + kFz * kFz, *u = c + kFz;   // scratch after C^-1
        double delta = c[r];
        for (int q = 0; q < r; ++q) {
            double t = 0.0;
            for (int k = 0; k < r; ++k) t += v.Cri[q * kFz + k] * c[k];
            u[q] = t;
            delta -= c[q] * t;
        }
        const double id = 1.0 / delta;
        u[kFz] = delta;   // for the update of z below
        for (int q = 0; q < r; ++q) {
            for (int k = 0; k < r; ++k) v.Cri[q * kFz + k] += u[q] * u[k] * id;
            v.Cri[q * kFz + r] = -u[q] * id;
            v.Cri[r * kFz + q] = -u[q] * id;
        }
        v.Cri[r * kFz + r] = id;
        v.Rp[r] = p;
    }
    __syncthreads();
    if (upd_z) {
        const double *u = v.Cri + kFz * kFz + kFz;
        const double f = v.z[p] / u[kFz];
        __syncthreads();   // every thread holds z_p before any position is written
        for (int i = threadIdx.x; i < s; i += kT) {
            double h = v.U[(size_t)r * v.m_cap + i];
            for (int q = 0; q < r; ++q) h -= v.U[(size_t)q * v.m_cap + i] * u[q];
            v.z[i] -= h * f;
        }
        __syncthreads();
        // frozen positions (the earlier ones and p) stay exactly zero
        if ((int)threadIdx.x <= r) v.z[v.Rp[threadIdx.x]] = 0.0;
        __syncthreads();
    }
    SUB(9);
    v.r = r + 1;
}

template <typename TG>
__device__ __forceinline__ void frozen_factors(Sv<TG> &v) {
    const int r = v.r, s = v.s;
    for (int i = threadIdx.x; i < s; i += kT) {
        double w[kFz];
#pragma unroll
        for (int q = 0; q < kFz; ++q) w[q] = q < r ? v.U[(size_t)q * v.m_cap + i] : 0.0;
        for (int q = 0; q < r; ++q) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < kFz; ++k) t += (k < r ? v.Cri[q * kFz + k] : 0.0) * w[k];
            v.V[(size_t)q * v.m_cap + i] = -t;
        }
    }
    __syncthreads();
}

// Drop the frozen positions (their rows and columns of H are zero once the
// downdate is applied) in descending order, each hole taking the last live
// position.
template <typename TG>
__device__ __forceinline__ void drop_frozen(Sv<TG> &v) {
    const int r = v.r;
    for (int n = 0; n < r; ++n) {
        int best = -1;
        for (int q = 0; q < r; ++q) best = max(best, v.Rp[q]);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int q = 0; q < r; ++q)
                if (v.Rp[q] == best) { v.Rp[q] = -1; break; }
        __syncthreads();
        drop_position(v, best);
    }
    v.r = 0;
    v.fz = 0;
}

// z += sum_p u_p (column p of the effective inverse H - W C^-1 W') over the
// positions p with u_p != 0 (right-hand sides moved by u_p), then u_p = 0:
// the update for all of them in one pass over their rows of H. Returns their
// number. The position list goes to v.rhs (free between solves).
template <typename TG>
__device__ __forceinline__ int heff_axpy_all(Sv<TG> &v, Red &red) {
    const int s = v.s, r = v.r;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int nf = 0;
    for (int i0 = 0; i0 < s; i0 += kT) {
        const int i = i0 + threadIdx.x;
        const bool on = i < s && v.u[i] != 0.0;
        const unsigned long long bal = __ballot(on);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) red.i[wid] = __popcll(bal);
        __syncthreads();
        int wbase = 0, tot = 0;
        for (int w = 0; w < kW; ++w) {
            if (w < wid) wbase += red.i[w];
            tot += red.i[w];
        }
        __syncthreads();
        if (on) v.rhs[nf + wbase + pre] = (double)i;
        nf += tot;
    }
    __syncthreads();
    if (nf == 0) return 0;
    // T = C^-1 (sum_p u_p W[., p]) for the frozen correction
    double T[kFz];
    {
        double wsum[kFz];
#pragma unroll
        for (int q = 0; q < kFz; ++q) wsum[q] = 0.0;
        for (int j = threadIdx.x; j < nf; j += kT) {
            const int p = (int)v.rhs[j];
            const double d = v.u[p];
#pragma unroll
            for (int q = 0; q < kFz; ++q)
                if (q < r) wsum[q] += d * v.U[(size_t)q * v.m_cap + p];
        }
        if (r > 0) bsum_vec<kFz>(wsum, red);
#pragma unroll
        for (int q = 0; q < kFz; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < kFz; ++k) acc += (q < r && k < r) ? v.Cri[q * kFz + k] * wsum[k] : 0.0;
            T[q] = acc;
        }
    }
    for (int i = threadIdx.x; i < s; i += kT) {
        double acc = 0.0;
        int j = 0;
        for (; j + 4 <= nf; j += 4) {
            double h[4], d[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = (int)v.rhs[j + e];
                h[e] = v.H[(size_t)p * v.ldh + i];
                d[e] = v.u[p];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) acc += d[e] * h[e];
        }
        for (; j < nf; ++j) {
            const int p = (int)v.rhs[j];
            acc += v.u[p] * v.H[(size_t)p * v.ldh + i];
        }
        for (int q = 0; q < r; ++q) acc -= v.U[(size_t)q * v.m_cap + i] * T[q];
        v.z[i] += acc;
    }
    v.bytes += 8.0 * (double)s * nf;
    __syncthreads();
    // frozen positions stay exactly zero; the moved right-hand sides are used
    if ((int)threadIdx.x < r) v.z[v.Rp[threadIdx.x]] = 0.0;
    for (int j = threadIdx.x; j < nf; j += kT) v.u[(int)v.rhs[j]] = 0.0;
    __syncthreads();
    return nf;
}

// Apply the frozen set to H (one rank-r pass: H <- H - W' C^-1 W) and drop
// the frozen positions from the active list.
template <typename TG>
__device__ __forceinline__ void compact(Sv<TG> &v, double *tile) {
    const int r = v.r;
    if (r == 0) return;
    const int s = v.s;
    v.bytes += 16.0 * (double)s * (double)s;
    SUB_START();
    frozen_factors(v);
    SUB(10);
    hupdate_all(v, s, r, tile);
    SUB(11);
    drop_frozen(v);
    SUB(12);
}

// Stage the frozen set as a deferred update instead of applying it: the
// next bordering block folds its rank into the pass that applies its own
// update (the frozen positions stay in the list, zero in beta and z, until
// that pass, and are dropped after it). With nothing to activate, the
// caller applies it with flush_pending.
template <typename TG>
__device__ __forceinline__ void stage_frozen(Sv<TG> &v) {
    if (v.r == 0 || v.pend != 0) return;
    frozen_factors(v);
    v.pend = v.r;
    v.fz = v.r;
}

// z = (inverse of the active block without the frozen positions) * in,
// with in and z zero at frozen positions.
template <typename TG>
__device__ __forceinline__ void solve_active(Sv<TG> &v, double *in, double *out, Red &red) {
    const int s = v.s, r = v.r;
    if (r > 0) {
        if ((int)threadIdx.x < r) in[v.Rp[threadIdx.x]] = 0.0;
        __syncthreads();
    }
    hgemv(v, in, out);
    if (r == 0) return;
    double t[kFz];
#pragma unroll
    for (int q = 0; q < kFz; ++q) t[q] = 0.0;
    for (int i = threadIdx.x; i < s; i += kT) {
        const double x = in[i];
#pragma unroll
        for (int q = 0; q < kFz; ++q)
            if (q < r) t[q] += v.U[(size_t)q * v.m_cap + i] * x;
    }
    bsum_vec<kFz>(t, red);
    double y[kFz];
#pragma unroll
    for (int q = 0; q < kFz; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kFz; ++k) acc += (q < r && k < r) ? v.Cri[q * kFz + k] * t[k] : 0.0;
        y[q] = acc;
    }
    for (int i = threadIdx.x; i < s; i += kT) {
        double acc = out[i];
#pragma unroll
        for (int q = 0; q < kFz; ++q)
            if (q < r) acc -= v.U[(size_t)q * v.m_cap + i] * y[q];
        out[i] = acc;
    }
    __syncthreads();
    if ((int)threadIdx.x < r) out[v.Rp[threadIdx.x]] = 0.0;
    __syncthreads();
}

// g = b - G beta - lambda2 beta over all coordinates (rows of the active
// set). Each thread owns one 16-byte group of adjacent coordinates (four
// FP32 or two FP64 Gram entries per load) and keeps sixteen Gram rows in
// flight: the pass is bound by bytes in flight per CU.
template <typename TG> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };

// Rows [r0, r1) of the active list Sl (beta by coordinate in bl): with
// Part, out_m = -sum_i G[Sl_i][m] bl[Sl_i] (a member's partial sum);
// otherwise out_m = b_m - lambda2 beta_m - sum_i G[Sl_i][m] bl[Sl_i].
template <bool Part, typename TG>
__device__ __forceinline__ void grad_rows(Sv<TG> &v, const int *Sl, const double *bl, int r0, int r1,
                                          double *out) {
    constexpr int kRows = 16;
    constexpr int VW = 16 / (int)sizeof(TG);
    using V = typename Vec16<TG>::type;
    const int M = v.M;
    const int ncol = (M + VW - 1) / VW;
    const size_t ldv = (size_t)v.mpad / VW;   // mpad is a multiple of 64
    for (int cb = threadIdx.x; cb < ncol; cb += kT) {
        const int m0 = cb * VW;
        double acc[VW];
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            const int m = m0 + c;
            acc[c] = (!Part && m < M) ? v.b[m] - v.l2 * bl[m] : 0.0;
        }
        const V *col = reinterpret_cast<const V *>(v.G + m0);
        int i = r0;
        for (; i + kRows <= r1; i += kRows) {
            V gv[kRows];
            double bb[kRows];
#pragma unroll
            for (int e = 0; e < kRows; ++e) {
                const int k = Sl[i + e];
                gv[e] = col[(size_t)k * ldv];
                bb[e] = bl[k];
            }
#pragma unroll
            for (int e = 0; e < kRows; ++e) {
                const TG *g = reinterpret_cast<const TG *>(&gv[e]);
#pragma unroll
                for (int c = 0; c < VW; ++c) acc[c] -= (double)g[c] * bb[e];
            }
        }
        for (; i < r1; ++i) {
            const int k = Sl[i];
            const V gv = col[(size_t)k * ldv];
            const TG *g = reinterpret_cast<const TG *>(&gv);
            const double bk = bl[k];
#pragma unroll
            for (int c = 0; c < VW; ++c) acc[c] -= (double)g[c] * bk;
        }
#pragma unroll
        for (int c = 0; c < VW; ++c)
            if (m0 + c < M) out[m0 + c] = acc[c];
    }
    __syncthreads();
}

template <typename TG>
__device__ __forceinline__ void full_gradient(Sv<TG> &v) {
    const int s = v.s, M = v.M;
    v.bytes += (double)s * M * sizeof(TG);
    if (!team_on(v)) {
        SUB_START();
        grad_rows<false>(v, v.S, v.beta, 0, s, v.g);
        SUB(13);
        return;
    }
    int *Sg = v.Sg();
    double *bco = v.bco();
    for (int i = threadIdx.x; i < s; i += kT) Sg[i] = v.S[i];
    for (int m = threadIdx.x; m < M; m += kT) bco[m] = v.beta[m];
    team_post(v, OP_GRAD, s, M);
    team_slice(v, OP_GRAD, s, M, 0, nullptr);
    team_join(v, OP_GRAD, s, M, nullptr);
    const size_t lp = (size_t)kB * v.m_cap;
    for (int m = threadIdx.x; m < M; m += kT) {
        double acc = v.part[m];
        for (int k = 1; k < v.T; ++k) acc += v.part[k * lp + m];
        v.g[m] = (v.b[m] - v.l2 * v.beta[m]) + acc;
    }
    __syncthreads();
}

// Activate the listed coordinates (blocked; single fallback on failure).
// Coordinates that cannot enter are deactivated. Returns false if none of a
// requested set could enter.
template <typename TG>
__device__ __forceinline__ bool activate(Sv<TG> &v, int *list, int n, Red &red, double *cinv, int *blk, double *tile,
                                         bool upd_z = false) {
    bool any = false;
    bool pre = false;   // this block's product came from the previous block's pass
    for (int b0 = 0; b0 < n; b0 += kB) {
        const int nb = min(kB, n - b0);
        if (threadIdx.x < nb) blk[threadIdx.x] = list[b0 + threadIdx.x];
        __syncthreads();
        // a full block followed by another shares its pass over H with it
        // (one workgroup only: the team's partial results hold kB columns);
        // a block followed by another defers its update
        const int nb_next = (!pre && nb == kB && b0 + nb < n && !team_on(v) && v.pend + 2 * kB <= kQ)
                                ? min(kB, n - b0 - nb) : 0;
        if (add_block(v, blk, nb, red, cinv, tile, upd_z, b0 + nb < n, list + b0 + nb, nb_next, pre)) {
            any = true;
            pre = nb_next > 0;
            continue;
        }
        pre = false;
        for (int q = 0; q < nb; ++q) {
            const int k = list[b0 + q];
            if (threadIdx.x == 0) blk[0] = k;
            __syncthreads();
            if (add_block(v, blk, 1, red, cinv, tile, upd_z)) {
                any = true;
            } else if (threadIdx.x == 0) {
                v.th[k] = 0;
                v.beta[k] = 0.0;
            }
            __syncthreads();
        }
    }
    flush_pending(v, tile);
    return any;
}

// Rebuild the inverse of the active block from the Gram: the frozen set is
// applied, the active coordinates are collected in position order and enter
// an empty block again by bordering (kB at a time). Used when a violating
// coordinate can no longer enter because the incrementally updated inverse
// has lost accuracy (ill-conditioned blocks after many updates). Signs are
// kept; coordinates that cannot re-enter are deactivated.
template <typename TG>
__device__ __forceinline__ void rebuild(Sv<TG> &v, int *list, Red &red, double *cinv, int *blk,
                                        double *tile) {
    compact(v, tile);
    const int s = v.s;
    for (int i = threadIdx.x; i < s; i += kT) v.rhs[i] = (double)v.S[i];
    __syncthreads();
    for (int i = threadIdx.x; i < s; i += kT) v.pos[v.S[i]] = -1;
    __syncthreads();
    v.s = 0;
    for (int b0 = 0; b0 < s; b0 += kInit) {
        const int nb = min(kInit, s - b0);
        if (threadIdx.x < nb) list[threadIdx.x] = (int)v.rhs[b0 + threadIdx.x];
        __syncthreads();
        activate(v, list, nb, red, cinv, blk, tile);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- FP64 phase
// Low-precision Gram modes: the first pass of the iteration solves the
// problem whose design and Gram are rounded to FP32 (or BF16). A second pass
// of the same iteration then finishes the FP64 problem from that point:
// gradients come from the Shepard-normalized FP64 design W64, recomputed
// from (x, c, sigma) for every product (nothing of it is stored), and the
// active solve (G64_SS + lambda2 I) z = b64_S - lambda1 theta_S is done by
// conjugate gradients preconditioned with H, which keeps being the inverse of
// the low-precision active block. The returned KKT residual certifies the
// FP64 problem.
struct Pol {
    const double *x, *y, *c, *sg;
    int N, dim;
    double *w;            // [M] -1 / (2 sigma_m^2)
    double *p, *q, *t;    // [m_cap] CG vectors by active position
    double *u;            // [N] per-sample vector
    double *is;           // [N] 1 / s_j (1 for the plain basis)
    int plain;            // unnormalized basis: W64 = Phi
    double *W;            // [M][npad] the FP64 design W64, built once per FP64 phase
    int ldw;              // npad
};

// Per-sample pass: for samples j (two per thread at a time, for independent
// exponentials in flight) over the centers k(i), i < n:
// sum_i phi_{j,k(i)} and sum_i phi_{j,k(i)} p_i.
template <typename K, typename F>
__device__ __forceinline__ void sample_pass(const Pol &P, int n, K key, const double *p, F out) {
    for (int j0 = threadIdx.x; j0 < P.N; j0 += 2 * kT) {
        const int j1 = min(j0 + kT, P.N - 1);
        double x0[3], x1[3];   // unused dimensions are zero on both sides
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x0[a] = a < P.dim ? P.x[(size_t)j0 * P.dim + a] : 0.0;
            x1[a] = a < P.dim ? P.x[(size_t)j1 * P.dim + a] : 0.0;
        }
        double s0 = 0.0, n0 = 0.0, s1 = 0.0, n1 = 0.0;
        for (int i = 0; i < n; ++i) {
            const int m = key(i);
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ca = a < P.dim ? P.c[(size_t)m * P.dim + a] : 0.0;
                d0 += (x0[a] - ca) * (x0[a] - ca);
                d1 += (x1[a] - ca) * (x1[a] - ca);
            }
            const double w = P.w[m], pv = p[i];
            const double f0 = exp(d0 * w), f1 = exp(d1 * w);
            s0 += f0;
            n0 += f0 * pv;
            s1 += f1;
            n1 += f1 * pv;
        }
        out(j0, s0, n0);
        if (j0 + kT < P.N) out(j0 + kT, s1, n1);
    }
    __syncthreads();
}

// Per-center pass: for items i < n (center k(i)), four per thread at a time,
// over all samples: sum_j phi_{j,k(i)} u_j.
template <typename K, typename F>
__device__ __forceinline__ void center_pass(const Pol &P, int n, K key, F out) {
    constexpr int R = 4;
    for (int i0 = threadIdx.x; i0 < n; i0 += R * kT) {
        double c[R][3], w[R], acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = key(min(i0 + r * kT, n - 1));
#pragma unroll
            for (int a = 0; a < 3; ++a) c[r][a] = a < P.dim ? P.c[(size_t)m * P.dim + a] : 0.0;
            w[r] = P.w[m];
            acc[r] = 0.0;
        }
        for (int j = 0; j < P.N; ++j) {
            double xj[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) xj[a] = a < P.dim ? P.x[(size_t)j * P.dim + a] : 0.0;
            const double uj = P.u[j];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double d = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) d += (xj[a] - c[r][a]) * (xj[a] - c[r][a]);
                acc[r] += exp(d * w[r]) * uj;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (i0 + r * kT < n) out(i0 + r * kT, acc[r]);
    }
    __syncthreads();
}

// The FP64 design W64[m][j] = phi_{j,m} / s_j (phi itself for the plain
// basis) for all m < M, j < N: one exponential per entry, built once when the
// FP64 phase starts; every later product streams it.
template <typename TG>
__device__ __forceinline__ void build_w64(Sv<TG> &v, const Pol &P, double *tile) {
    // W64[m][j] = phi_mj / sum_k phi_kj: per sample j the sum over all M
    // centers first, then the normalized entries written once (the
    // exponentials are recomputed, the same values in the same order); the
    // centers and widths are staged in LDS in chunks of kCW
    constexpr int kCW = 512;
    static_assert(4 * kCW <= kQ * kTile, "center staging fits the tile");
    double *scx = tile, *sw = tile + 3 * kCW;
    const int M = v.M;
    v.bytes += 8.0 * (double)M * (double)P.N;
    for (int j0 = 0; j0 < P.N; j0 += kT) {
        const int j = j0 + threadIdx.x;
        const bool live = j < P.N;
        double xj[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) xj[a] = (live && a < P.dim) ? P.x[(size_t)j * P.dim + a] : 0.0;
        double is = 1.0;
        for (int pass = P.plain ? 1 : 0; pass < 2; ++pass) {
            double sj = 0.0;
            for (int m0 = 0; m0 < M; m0 += kCW) {
                const int cnt = min(kCW, M - m0);
                __syncthreads();
                for (int t = threadIdx.x; t < cnt; t += kT) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) scx[t * 3 + a] = a < P.dim ? P.c[(size_t)(m0 + t) * P.dim + a] : 0.0;
                    sw[t] = P.w[m0 + t];
                }
                __syncthreads();
                if (!live) continue;
                for (int t = 0; t < cnt; ++t) {
                    double d = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) d += (xj[a] - scx[t * 3 + a]) * (xj[a] - scx[t * 3 + a]);
                    const double f = exp(d * sw[t]);
                    if (pass == 0) sj += f;
                    else P.W[(size_t)(m0 + t) * P.ldw + j] = P.plain ? f : f * is;
                }
            }
            if (pass == 0) is = 1.0 / sj;
        }
        if (live) P.is[j] = is;
    }
    __syncthreads();
}

// t_j = sum_{i < n} W64[key(i)][j] p_i for every sample j (threads over j,
// two samples per thread and eight rows in flight for each; every row read
// coalesced).
template <typename K>
__device__ __forceinline__ void w_combine(const Pol &P, int n, K key, const double *p, double *t) {
    for (int j0 = threadIdx.x; j0 < P.N; j0 += 2 * kT) {
        const int j1 = j0 + kT;
        const bool two = j1 < P.N;
        const int j1c = two ? j1 : j0;
        double acc0 = 0.0, acc1 = 0.0;
        int i = 0;
        for (; i + 8 <= n; i += 8) {
            double w0[8], w1[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double *row = P.W + (size_t)key(i + e) * P.ldw;
                w0[e] = row[j0];
                w1[e] = row[j1c];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                acc0 += w0[e] * p[i + e];
                acc1 += w1[e] * p[i + e];
            }
        }
        for (; i < n; ++i) {
            const double *row = P.W + (size_t)key(i) * P.ldw;
            acc0 += row[j0] * p[i];
            acc1 += row[j1c] * p[i];
        }
        t[j0] = acc0;
        if (two) t[j1] = acc1;
    }
    __syncthreads();
}

// out(i, sum_j W64[key(i)][j] u_j) for i < n: each wave takes four rows at a
// time, the lanes over j (eight loads in flight per lane), then a wave
// reduction per row.
template <typename K, typename F>
__device__ __forceinline__ void w_dot(const Pol &P, int n, K key, const double *u, F out) {
    constexpr int RW = 4;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i0 = wid * RW; i0 < n; i0 += kW * RW) {
        const double *row[RW];
        double acc[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            row[r] = P.W + (size_t)key(min(i0 + r, n - 1)) * P.ldw;
            acc[r] = 0.0;
        }
        int j = lane;
        for (; j + 64 < P.N; j += 128) {
            const double u0 = u[j], u1 = u[j + 64];
            double a[RW], b[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) { a[r] = row[r][j]; b[r] = row[r][j + 64]; }
#pragma unroll
            for (int r = 0; r < RW; ++r) acc[r] += a[r] * u0 + b[r] * u1;
        }
        if (j < P.N) {
            const double u0 = u[j];
#pragma unroll
            for (int r = 0; r < RW; ++r) acc[r] += row[r][j] * u0;
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, 64);
        }
        if (lane == 0)
#pragma unroll
            for (int r = 0; r < RW; ++r)
                if (i0 + r < n) out(i0 + r, acc[r]);
    }
    __syncthreads();
}

// The residual e_j = y_j - (W64 beta)_j over the active coordinates, then
// g_m = (W64' e)_m - lambda2 beta_m for every m < M.
template <typename TG>
__device__ __forceinline__ void grad64(Sv<TG> &v, const Pol &P) {
    const int *S = v.S;
    const double *beta = v.beta;
    v.bytes += 8.0 * (double)(v.s + v.M) * (double)P.N;
    // active coordinates carry all of W64 beta (beta is zero elsewhere);
    // p_i = beta at position i, staged in P.t
    for (int i = threadIdx.x; i < v.s; i += kT) P.t[i] = beta[S[i]];
    __syncthreads();
    w_combine(P, v.s, [S](int i) { return S[i]; }, P.t, P.u);
    for (int j = threadIdx.x; j < P.N; j += kT) P.u[j] = P.y[j] - P.u[j];
    __syncthreads();
    w_dot(P, v.M, [](int i) { return i; }, P.u, [&](int m, double acc) { v.g[m] = acc - v.l2 * beta[m]; });
}

// q = (W64_S' W64_S + lambda2 I) p over active positions.
template <typename TG>
__device__ __forceinline__ void apply64(Sv<TG> &v, const Pol &P, const double *p, double *q) {
    const int *S = v.S;
    v.bytes += 16.0 * (double)v.s * (double)P.N;
    w_combine(P, v.s, [S](int i) { return S[i]; }, p, P.u);
    w_dot(P, v.s, [S](int i) { return S[i]; }, P.u, [&](int i, double acc) { q[i] = acc + v.l2 * p[i]; });
}

// z (by position) solves the FP64 reduced system on the signed active set,
// by CG from beta_S whose residual g_S - lambda1 theta_S needs the FP64
// gradient at beta in v.g. No frozen positions may be pending. Returns the
// number of products with the FP64 block.
template <typename TG>
__device__ __forceinline__ int cg64(Sv<TG> &v, const Pol &P, Red &red, double tol, double *z) {
    const int s = v.s;
    double *r = v.rhs;
    double rm = 0.0;
    for (int i = threadIdx.x; i < s; i += kT) {
        const int k = v.S[i];
        z[i] = v.beta[k];
        r[i] = v.g[k] - v.l1 * (double)v.th[k];
        rm = fmax(rm, fabs(r[i]));
    }
    if (bmax(rm, red) <= tol) return 0;
    solve_active(v, r, P.t, red);
    double rz = 0.0;
    for (int i = threadIdx.x; i < s; i += kT) {
        P.p[i] = P.t[i];
        rz += r[i] * P.t[i];
    }
    rz = bsum(rz, red);
    int it = 0;
    while (it < kPolishMax) {
        apply64(v, P, P.p, P.q);
        ++it;
        double pq = 0.0;
        for (int i = threadIdx.x; i < s; i += kT) pq += P.p[i] * P.q[i];
        pq = bsum(pq, red);
        if (!(pq > 0.0) || !(rz > 0.0)) break;
        const double al = rz / pq;
        double rmx = 0.0;
        for (int i = threadIdx.x; i < s; i += kT) {
            z[i] += al * P.p[i];
            r[i] -= al * P.q[i];
            rmx = fmax(rmx, fabs(r[i]));
        }
        if (bmax(rmx, red) <= tol) break;
        solve_active(v, r, P.t, red);
        double rzn = 0.0;
        for (int i = threadIdx.x; i < s; i += kT) rzn += r[i] * P.t[i];
        rzn = bsum(rzn, red);
        const double bt = rzn / rz;
        rz = rzn;
        for (int i = threadIdx.x; i < s; i += kT) P.p[i] = P.t[i] + bt * P.p[i];
        __syncthreads();
    }
    return it;
}

// Member k's rows of a posted pass: inputs from the team buffers and the
// bordering rows, results to its partial block (or to its rows of H).
template <typename TG>
__device__ __forceinline__ void team_slice(Sv<TG> &v, int op, int s, int n, int k, double *tile) {
    const int r0 = team_row0(k, s, v.T), r1 = team_row0(k + 1, s, v.T);
    double *mine = v.part + (size_t)k * kB * v.m_cap;
    if (op == OP_GEMV) hgemv_rows(v, v.xin(), mine, r0, r1);
    else if (op == OP_UPASS) upass(v, n, r0, r1, mine, tile);
    else if (op == OP_UPDATE) hupdate_rows(v, s, n, tile, r0, r1);
    else if (op == OP_GRAD) grad_rows<true>(v, v.Sg(), v.bco(), r0, r1, mine);
}

// Members other than the leader: take row slices of the leader's passes
// until it quits, or leave (marked kGone) after a bounded wait for the next
// command.
template <typename TG>
__device__ __forceinline__ void team_serve(Sv<TG> &v, int rank, double *tile) {
    unsigned long long seen = 0;   // meaningful in thread 0
    for (;;) {
        if (threadIdx.x == 0) {
            const long long t0 = wall_clock64();
            unsigned long long c;
            while ((c = ld_relaxed(&v.ctl[0])) == seen) {
                if (wall_clock64() - t0 > v.idle) break;
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (c == seen) {
                __hip_atomic_store(&v.ctl[16 * rank], kGone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                v.tsh[0] = (unsigned)OP_QUIT;
            } else {
                v.tsh[0] = (unsigned)v.ctl[1];
            }
            v.tsh[1] = (unsigned)v.ctl[2];
            v.tsh[2] = (unsigned)v.ctl[3];
            seen = c;
        }
        __syncthreads();
        const int op = (int)v.tsh[0], s = (int)v.tsh[1], n = (int)v.tsh[2];
        __syncthreads();
        if (op < OP_GEMV || op > OP_GRAD) return;
        v.s = s;
        team_slice(v, op, s, n, rank, tile);
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&v.ctl[16 * rank], seen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename TG>
__device__ __forceinline__ void solve_one(const FitArgs &a, Sv<TG> &v, int s_id, double *sc,
                                          const int32_t *__restrict__ flags, Red &red, double *cinv, int *blk,
                                          int *list, double *tile);

// kTeam = false: one workgroup per subdomain, no team code compiled in
// (T is the constant 1, every team branch folds away). kVG: the iteration's
// per-center vectors live in the subdomain's scratch in HBM instead of LDS
// (dictionaries too large for LDS; one workgroup per subdomain).
template <typename TG, bool kTeam, bool kVG = false>
__global__ void __launch_bounds__(kT)
k_solve(FitArgs a, const TG *__restrict__ Gall, double *__restrict__ Hall,
        double *__restrict__ scratch, const int32_t *__restrict__ flags, unsigned long long *__restrict__ tctl) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    __shared__ Red red;
    __shared__ double cinv[kB * kB];
    __shared__ int blk[kB];
    __shared__ int list[kAdd > kInit ? kAdd : kInit];
    __shared__ double tile[kQ * kTile];
    __shared__ int frz[kFz];
    __shared__ double cri[kFz * kFz + 3 * kFz + 1];
    __shared__ unsigned tsh[5];
#ifdef PAM_PHASE_PROFILE
    __shared__ long long sp[24];
    if (threadIdx.x < 24) sp[threadIdx.x] = 0;
#endif
    // Workgroups are dispatched to the 8 XCDs round robin (block b to XCD
    // b mod 8): a team takes T blocks of one XCD (shared L2 for its partial
    // results) and the leaders spread evenly over all XCDs. With T = 1 this
    // is the identity; with T > 1 the grid is padded to whole groups of 8.
    const int T = (kTeam && a.team > 1) ? a.team : 1;
    const int xcd = (int)blockIdx.x & 7, w = (int)blockIdx.x >> 3;
    const int loc = xcd + 8 * (w / T), rank = w - (w / T) * T;
    if (loc >= a.sub_count) return;
    const int s_id = a.sub_begin + loc;
    if (a.active && !a.active[s_id]) return;   // the whole team
    Sv<TG> v;
    v.G = Gall + (size_t)loc * a.mpad * a.mpad;
    v.mpad = a.mpad;
    v.M = max(0, min(a.m[s_id], a.m_cap));
    v.m_cap = a.m_cap;
    v.ldh = ldh_of(a.m_cap);
    v.l1 = a.lambda1_sub ? a.lambda1_sub[s_id] : a.lambda1;
    v.l2 = a.lambda2_sub ? a.lambda2_sub[s_id] : a.lambda2;
    v.H = Hall + (size_t)loc * h_elems_of(a.m_cap);
    double *sc = scratch + (size_t)loc * scratch_elems_of(a.m_cap, a.npad, a.precision, T, kVG);
    v.Ag = sc;
    v.U = sc + (size_t)kQ * a.m_cap;
    v.V = sc + (size_t)2 * kQ * a.m_cap;
    const int Mc = (int)round_up(a.m_cap, 8);
    double *ld = kVG ? sc + scratch_elems_of(a.m_cap, a.npad, a.precision, T, false)
                     : reinterpret_cast<double *>(lds_raw);
    v.g = ld;
    v.beta = ld + Mc;
    v.z = ld + 2 * Mc;
    v.rhs = ld + 3 * Mc;
    v.u = ld + 4 * Mc;
    v.b = ld + 5 * Mc;
    v.S = reinterpret_cast<int *>(ld + 6 * Mc);
    v.pos = v.S + Mc;
    v.th = reinterpret_cast<signed char *>(v.pos + Mc);
    v.s = 0;
    v.bytes = 0.0;
    v.r = 0;
    v.pend = 0;
    v.fz = 0;
    v.Rp = frz;
    v.Cri = cri;
    v.T = T;
    v.team_min = a.team_min;
    v.idle = a.team_idle_us > 0 ? (long long)a.team_idle_us * 100 : kTeamWait;   // 100 MHz clock
    v.tsh = tsh;
#ifdef PAM_PHASE_PROFILE
    v.sp = sp;
#endif
    v.ctl = nullptr;
    v.part = nullptr;
    if (threadIdx.x < 5) tsh[threadIdx.x] = 0;
    __syncthreads();
    if (T > 1) {
        v.ctl = tctl + (size_t)loc * kCtl;
        v.part = sc + scratch_elems_of(a.m_cap, a.npad, a.precision, 1);
        if (rank > 0) {
            team_serve(v, rank, tile);
            return;
        }
    }
    solve_one(a, v, s_id, sc, flags, red, cinv, blk, list, tile);
    if (T > 1) team_post(v, OP_QUIT, 0, 0);   // also after a failure: members still waiting exit
}

template <typename TG>
__device__ __forceinline__ void solve_one(const FitArgs &a, Sv<TG> &v, int s_id, double *sc,
                                          const int32_t *__restrict__ flags, Red &red, double *cinv, int *blk,
                                          int *list, double *tile) {
    const int M = v.M;
#ifdef PAM_PHASE_PROFILE
    long long ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long ph_last = wall_clock64();
    double phb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double phb_last = 0.0;
    int n_rm = 0, n_add = 0, n_ls = 0, n_cons = 0, it_ex0 = 0;
    long long t_ex0 = 0;
#endif
    double *beta_out = a.beta + (size_t)s_id * a.m_cap;
    pam_fit_stats *st = a.stats ? a.stats + s_id : nullptr;
    const long long t_begin = wall_clock64();   // the 100 MHz constant clock

    if ((flags[s_id] & 3) || M <= 0 || a.off[s_id + 1] <= a.off[s_id]) {
        for (int m = threadIdx.x; m < a.m_cap; m += kT) beta_out[m] = 0.0;
        if (st && threadIdx.x == 0) {
            // non-finite input first; then no centers or no samples is EMPTY
            // (the empty design also flags underflow)
            const bool empty = M <= 0 || a.off[s_id + 1] <= a.off[s_id];
            st->status = (flags[s_id] & 2) ? PAM_ST_NONFINITE : empty ? PAM_ST_EMPTY : PAM_ST_UNDERFLOW;
            st->cd_sweeps = 0; st->iters = 0; st->support = 0; st->kkt = 0.0;
            st->stream_bytes = 0.0; st->polish = 0; st->team = 1; st->solve_us = 0.0;
        }
        return;
    }
    // ---- start point and gradient
    for (int m = threadIdx.x; m < M; m += kT) {
        v.beta[m] = a.warm_start ? beta_out[m] : 0.0;
        v.pos[m] = -1;
        v.b[m] = Gat(v, m, M);
        v.g[m] = v.b[m];
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += kT) v.g[m] -= v.l2 * v.beta[m];
    if (a.warm_start) {
        for (int k = 0; k < M; ++k) {
            const double bk = v.beta[k];
            if (bk == 0.0) continue;
            for (int m = threadIdx.x; m < M; m += kT) v.g[m] -= (double)v.G[(size_t)k * v.mpad + m] * bk;
        }
    }
    __syncthreads();
    PHASE_MARK(0);
    // ---- cyclic coordinate descent warm-up, creation order
    int sweeps = 0;
    // warm starts (previous round, caller's point) go straight to the
    // active-set iteration: CD from a good point only densifies the support
    // and a support hint (cold fits only) replaces the warm-up
    const uint8_t *hint = (a.hint && !a.warm_start) ? a.hint + (size_t)s_id * a.m_cap : nullptr;
    const int cd_sweeps = (a.warm_start || hint) ? 0 : a.cd_sweeps;
    if (cd_sweeps > 0) {
        // diagonal of the Gram + lambda2 in LDS (u is free until the active set)
        for (int m = threadIdx.x; m < M; m += kT) v.u[m] = Gat(v, m, m) + v.l2;
        __syncthreads();
    }
    for (; sweeps < cd_sweeps; ++sweeps) {
        double dmax = 0.0;
        for (int m = 0; m < M; ++m) {
            const double amm = v.u[m];
            const double bm = v.beta[m];
            const double zz = v.g[m] + amm * bm;
            const double az = fabs(zz) - v.l1;
            const double nb = az > 0.0 ? sgn(zz) * az / amm : 0.0;
            const double d = nb - bm;
            if (d != 0.0) {
                dmax = fmax(dmax, fabs(d));
                v.bytes += (double)M * sizeof(TG);
                __syncthreads();   // every thread has read g_m and beta_m
                for (int k = threadIdx.x; k < M; k += kT) {
                    double gk = v.g[k] - (double)v.G[(size_t)m * v.mpad + k] * d;
                    if (k == m) {
                        gk -= v.l2 * d;
                        v.beta[m] = nb;
                    }
                    v.g[k] = gk;
                }
                __syncthreads();
            }
        }
        if (dmax == 0.0) { ++sweeps; break; }
    }
    PHASE_MARK(1);
    // ---- signed active set from the start point (and the support hint)
    for (int m = threadIdx.x; m < M; m += kT) {
        int t = (int)sgn(v.beta[m]);
        if (t == 0 && hint && hint[m]) t = (int)sgn(v.g[m]);
        v.th[m] = (signed char)t;
    }
    __syncthreads();
    // initial active block, ascending coordinate order, kInit at a time (three
    // bordering blocks whose updates go to H in one rank-24 pass)
    for (int m0 = 0; m0 < M; m0 += kT) {
        const int m = m0 + threadIdx.x;
        const bool on = m < M && v.th[m] != 0;
        // compact this chunk in order with a block scan of the flags
        const unsigned long long bal = __ballot(on);
        const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) red.i[wid] = __popcll(bal);
        __syncthreads();
        int wbase = 0, tot = 0;
        for (int w = 0; w < kW; ++w) {
            if (w < wid) wbase += red.i[w];
            tot += red.i[w];
        }
        __syncthreads();
        if (on) v.rhs[wbase + pre] = (double)m;   // rhs is free here
        __syncthreads();
        for (int b0 = 0; b0 < tot; b0 += kInit) {
            const int nb = min(kInit, tot - b0);
            if (threadIdx.x < nb) list[threadIdx.x] = (int)v.rhs[b0 + threadIdx.x];
            __syncthreads();
            activate(v, list, nb, red, cinv, blk, tile);
            __syncthreads();
        }
    }
    for (int m = threadIdx.x; m < M; m += kT)
        if (v.th[m] == 0) v.beta[m] = 0.0;
    __syncthreads();
    if (hint && v.s > 0) {
        // signs of the hinted set from the ridge solution on it (lambda1
        // dropped): near the minimizer's support these are its signs, which
        // the gradient at zero often is not
        for (int i = threadIdx.x; i < v.s; i += kT) v.rhs[i] = v.b[v.S[i]];
        __syncthreads();
        solve_active(v, v.rhs, v.z, red);
        for (int i = threadIdx.x; i < v.s; i += kT) {
            const int t = (int)sgn(v.z[i]);
            if (t != 0) v.th[v.S[i]] = (signed char)t;
        }
        __syncthreads();
    }
    full_gradient(v);
    PHASE_MARK(2);
#ifdef PAM_PHASE_PROFILE
    const int s_init = v.s;
#endif

    // ---- exact sign-consistent active-set iteration
    const double bnorm = bmax([&] {
        double t = 0.0;
        for (int m = threadIdx.x; m < M; m += kT) t = fmax(t, fabs(v.b[m]));
        return t;
    }(), red);
    int it = 0, status = PAM_ST_NOCONV, refines = 0, n_cg = 0, rebuilds = 0;
    bool skip_solve = false, ran_ex = false;
    // v.z holds the solution of the current signed block (zv): line searches
    // and activations then carry it by rank-one and bordering identities
    // instead of a pass over H; a full solve at least every kIncMax updates
    bool zv = false;
    int n_inc = 0;
#ifdef PAM_INC_CHECK
    int dbg_op = 0, dbg_n = 0;
#endif
    constexpr bool kLow = sizeof(TG) < sizeof(double);
    Pol P{};
    if (kLow) {
        const int64_t j0 = a.off[s_id];
        P.x = a.x + (size_t)j0 * a.dim;
        P.y = a.y + j0;
        P.c = a.c + (size_t)s_id * a.m_cap * a.dim;
        P.sg = a.sigma + (size_t)s_id * a.m_cap;
        P.N = (int)(a.off[s_id + 1] - j0);
        P.dim = a.dim;
        P.w = sc + (size_t)3 * kQ * a.m_cap;
        P.p = P.w + a.m_cap;
        P.q = P.p + a.m_cap;
        P.t = P.q + a.m_cap;
        P.u = P.t + a.m_cap;
        P.plain = a.basis == PAM_BASIS_PLAIN;
        P.is = P.u + a.npad;
        P.W = P.is + a.npad;
        P.ldw = a.npad;
        for (int m = threadIdx.x; m < M; m += kT) P.w[m] = -0.5 / (P.sg[m] * P.sg[m]);
        __syncthreads();
    }
    // pass 0 solves the problem of the stored Gram; low-precision modes then
    // finish the FP64 problem from its end point (pass 1)
    for (int phase = 0; phase < (kLow ? 2 : 1); ++phase) {
    const bool ex = phase == 1;
    if (ex) {
        if (status != PAM_ST_OK) break;
        __syncthreads();
        compact(v, tile);
        SUB_START();
        build_w64(v, P, tile);
        SUB(20);
        grad64(v, P);
        SUB(21);
        status = PAM_ST_NOCONV;
        refines = 0;
        rebuilds = 0;
        skip_solve = false;
        ran_ex = true;
#ifdef PAM_PHASE_PROFILE
        it_ex0 = it;
        t_ex0 = wall_clock64();
#endif
    }
    // the FP64 gradient is a recomputed sum of N terms: its tolerances
    const double gtol = (ex ? 1e-12 : 1e-15) * fmax(1.0, bnorm);
    const double viol_tol = v.l1 * (1.0 + 1e-12) + (ex ? 1e-12 : 1e-14) * bnorm;
    // the FP64 pass starts next to the minimizer; a bound on its length
    // guards against cycling on margins at the FP64 rounding level
    const int it_end = ex ? min(a.max_iter, it + 2 * M + 100) : a.max_iter;
    while (it < it_end) {
        ++it;
        // a long run means sign decisions taken on an inverse that the many
        // incremental updates made inexact (ill-conditioned blocks): start
        // it afresh from the Gram at 4M and 8M iterations
        if (!ex && (it == 4 * M || it == 8 * M) && v.s > 0) {
            rebuild(v, list, red, cinv, blk, tile);
            zv = false;
            n_inc = 0;
            skip_solve = false;
        }
        if (v.s > 0 && !skip_solve) {
            SUB_START();
            if (ex) compact(v, tile);   // the CG solve runs on live positions only
            SUB(22);
            const int s = v.s;
            // full solve of the signed block into v.z
            auto solve_full = [&]() {
                for (int i = threadIdx.x; i < s; i += kT) {
                    const int k = v.S[i];
                    v.rhs[i] = v.b[k] - v.l1 * (double)v.th[k];
                }
                __syncthreads();
                solve_active(v, v.rhs, v.z, red);
                zv = true;
                n_inc = 0;
            };
            bool fresh = true;
            if (ex) {
                SUB_START();
                n_cg += cg64(v, P, red, gtol, v.z);
                SUB(19);
            } else if (zv && n_inc < kIncMax) {
                fresh = n_inc == 0;   // carried by the identities
#ifdef PAM_INC_CHECK
                {
                    for (int i = threadIdx.x; i < s; i += kT) {
                        const int k = v.S[i];
                        v.rhs[i] = v.b[k] - v.l1 * (double)v.th[k];
                    }
                    __syncthreads();
                    double *zf = v.Ag;
                    solve_active(v, v.rhs, zf, red);
                    double dm = 0.0, zm = 0.0;
                    int im = -1;
                    for (int i = threadIdx.x; i < s; i += kT) {
                        const double dd = fabs(zf[i] - v.z[i]);
                        if (dd > dm) { dm = dd; im = i; }
                        zm = fmax(zm, fabs(zf[i]));
                    }
                    VI xx; xx.v = dm; xx.i = im;
                    xx = bargmax(xx, red);
                    zm = bmax(zm, red);
                    if (threadIdx.x == 0 && xx.v > 1e-11 * zm && dbg_n < 8) {
                        printf("INC sub=%d it=%d s=%d r=%d n_inc=%d last_op=%d diff=%.3e at %d (zf %.3e z %.3e th %d) zmax=%.3e\n",
                               s_id, it, s, v.r, n_inc, dbg_op, xx.v, xx.i, zf[xx.i], v.z[xx.i], (int)v.th[v.S[xx.i]], zm);
                    }
                    if (xx.v > 1e-11 * zm) ++dbg_n;
                    __syncthreads();
                }
#endif
            } else {
                solve_full();
            }
            PHASE_MARK(3);
            bool mine = true;
            for (int i = threadIdx.x; i < s; i += kT)
                if ((int)sgn(v.z[i]) != v.th[v.S[i]]) mine = false;
            // the carried solution steers line searches; after more than
            // kConfirm updates a step is accepted as consistent only on a
            // solve of its own (the identities lose about eps * cond(G) per
            // update)
            if (!fresh && n_inc > kConfirm && ball(mine, red)) {
                solve_full();
                mine = true;
                for (int i = threadIdx.x; i < s; i += kT)
                    if ((int)sgn(v.z[i]) != v.th[v.S[i]]) mine = false;
            }
            if (!ball(mine, red)) {
                // discrete line search from beta_S to z over the zero crossings
                double p1 = 0.0, p2 = 0.0, p3 = 0.0;
                for (int i = threadIdx.x; i < s; i += kT) {
                    const int k = v.S[i];
                    const double b0 = v.beta[k], d = v.z[i] - b0;
                    p1 -= v.g[k] * d;
                    p2 += d * (v.g[k] - v.l1 * (double)v.th[k]);
                    p3 += fabs(v.z[i]) - fabs(b0);
                }
                double cc[3] = {p1, p2, p3};
                bsum_vec<3>(cc, red);
                const double c1 = cc[0], c2 = cc[1];
                double best_f = c1 + 0.5 * c2 + v.l1 * cc[2];   // t = 1
                double best_t = 1.0;
                // candidates in position order: compacted with a block scan
                for (int c0 = 0; c0 < s; c0 += kT) {
                    const int i = c0 + threadIdx.x;
                    double t = 2.0;
                    if (i < s) {
                        const double b0 = v.beta[v.S[i]], zi = v.z[i];
                        if (b0 != 0.0 && sgn(zi) != sgn(b0)) {
                            const double tt = b0 / (b0 - zi);
                            if (tt > 0.0 && tt < 1.0) t = tt;
                        }
                    }
                    const bool is_c = t < 1.0;
                    const unsigned long long bal = __ballot(is_c);
                    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
                    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
                    if (lane == 0) red.i[wid] = __popcll(bal);
                    __syncthreads();
                    int wbase = 0, tot = 0;
                    for (int w = 0; w < kW; ++w) {
                        if (w < wid) wbase += red.i[w];
                        tot += red.i[w];
                    }
                    __syncthreads();
                    if (is_c) v.u[wbase + pre] = t;      // u is free here
                    __syncthreads();
                    for (int q0 = 0; q0 < tot; q0 += kB) {
                        const int nq = min(kB, tot - q0);
                        double tq[kB], f[kB];
#pragma unroll
                        for (int q = 0; q < kB; ++q) {
                            tq[q] = q < nq ? v.u[q0 + q] : 0.0;
                            f[q] = 0.0;
                        }
                        for (int jq = threadIdx.x; jq < s; jq += kT) {
                            const double b0 = v.beta[v.S[jq]], d = v.z[jq] - b0;
                            const double ab0 = fabs(b0);
#pragma unroll
                            for (int q = 0; q < kB; ++q) f[q] += fabs(b0 + tq[q] * d) - ab0;
                        }
                        bsum_vec<kB>(f, red);
                        for (int q = 0; q < nq; ++q) {
                            const double fq = tq[q] * c1 + 0.5 * tq[q] * tq[q] * c2 + v.l1 * f[q];
                            if (fq < best_f) { best_f = fq; best_t = tq[q]; }
                        }
                    }
                }
                const double tstar = best_t;
                PHASE_MARK(4);
                SUB_START();
                for (int i = threadIdx.x; i < s; i += kT) {
                    const int k = v.S[i];
                    const double b0 = v.beta[k], zi = v.z[i];
                    double nb = b0 + tstar * (zi - b0);
                    if (tstar < 1.0 && b0 != 0.0 && sgn(zi) != sgn(b0) && b0 / (b0 - zi) == tstar) nb = 0.0;
                    const int t0 = v.th[k];
                    if (t0 == 0) nb = 0.0;   // a frozen position awaiting the downdate
                    v.g[k] -= tstar * (v.g[k] - v.l1 * (double)t0);
                    v.beta[k] = nb;
                    const int t1 = (int)sgn(nb);
                    // a coordinate that entered at zero may leave the line search
                    // with the other sign: its right-hand side moves by 2 lambda1 theta
                    v.u[i] = (t1 != 0 && t1 != t0) ? 2.0 * v.l1 * (double)t0 : 0.0;
                    v.th[k] = (signed char)t1;
                }
                __syncthreads();
                SUB(15);
                const bool inc = zv && !ex;
                if (inc) {
                    const int nf = heff_axpy_all(v, red);
                    n_inc += nf;
#ifdef PAM_INC_CHECK
                    if (nf > 0) dbg_op = (dbg_op % 1000) * 10 + 1;
#endif
                } else {
                    zv = false;
                }
                SUB(16);
                // freeze the coordinates that reached zero (batched downdate)
                // (every zero position not yet frozen, highest first; a full
                // frozen set is applied and the positions are collected again)
                for (;;) {
                    SUB_START();
                    int nz = 0;
                    {
                        const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
                        for (int p0 = 0; p0 < v.s; p0 += kT) {
                            const int p = p0 + threadIdx.x;
                            bool on = p < v.s && v.th[v.S[p]] == 0;
                            if (on)
                                for (int q = 0; q < v.r; ++q) on &= v.Rp[q] != p;
                            const unsigned long long bal = __ballot(on);
                            const int pre = __popcll(bal & ((1ull << lane) - 1ull));
                            if (lane == 0) red.i[wid] = __popcll(bal);
                            __syncthreads();
                            int wbase = 0, tot = 0;
                            for (int w = 0; w < kW; ++w) {
                                if (w < wid) wbase += red.i[w];
                                tot += red.i[w];
                            }
                            __syncthreads();
                            if (on) v.rhs[nz + wbase + pre] = (double)p;   // rhs is free here
                            nz += tot;
                        }
                        __syncthreads();
                    }
                    SUB(17);
                    bool moved = false;
                    for (int e = nz - 1; e >= 0; --e) {
                        if (v.r == kFz) {
                            compact(v, tile);
                            moved = true;   // positions moved: collect again
                            break;
                        }
                        freeze(v, (int)v.rhs[e], inc);
                        n_inc += inc ? 1 : 0;
#ifdef PAM_INC_CHECK
                        dbg_op = (dbg_op % 1000) * 10 + 2;
#endif
#ifdef PAM_PHASE_PROFILE
                        ++n_rm;
#endif
                    }
                    if (!moved) break;
                }
                PHASE_MARK(5);
#ifdef PAM_PHASE_PROFILE
                ++n_ls;
#endif
                refines = 0;   // the refinement budget counts consecutive attempts only
                continue;
            }
            for (int i = threadIdx.x; i < s; i += kT) v.beta[v.S[i]] = v.z[i];
            __syncthreads();
            // the frozen set's downdate rides on the next activation's update
            if (ex) compact(v, tile);
            else stage_frozen(v);
        }
        skip_solve = false;
        if (ex) grad64(v, P);
        else full_gradient(v);
        PHASE_MARK(6);
#ifdef PAM_PHASE_PROFILE
        ++n_cons;
#endif
        SUB_START();
        // worst inactive violations (up to kAdd, by |g| then index), bordered
        // kB at a time
        // (after many iterations: one activation per step). Each wave takes
        // its own best kAdd by repeated wave reductions, each pick the best
        // candidate ordered after the previous one; wave 0 then takes the
        // best of the waves' picks the same way: the same list, in the same
        // order, as kAdd block-wide reductions, with two barriers.
        const int kmax = it > 4 * M ? 1 : kAdd;
        int nadd = 0;
        {
            static_assert(kW * kAdd == 2 * 64, "the waves' picks are two per lane of one wave");
            const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
            double *cv = tile, *ci = tile + kW * kAdd;   // the waves' picks (tile is free here)
            double pv = INFINITY;
            int pi = -1;
            int r = 0;
            for (; r < kmax; ++r) {
                VI x; x.v = -1.0; x.i = -1;
                for (int m = lane + 64 * wid; m < M; m += kT) {
                    if (v.pos[m] >= 0) continue;
                    const double c = fabs(v.g[m]);
                    if (!(c < pv || (c == pv && m > pi))) continue;   // ordered after the last pick
                    VI cc; cc.v = c; cc.i = m;
                    x = vmax(x, cc);
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    VI y;
                    y.v = __shfl_xor(x.v, o, 64);
                    y.i = __shfl_xor(x.i, o, 64);
                    x = vmax(x, y);
                }
                if (x.i < 0 || x.v <= viol_tol) break;   // uniform over the wave
                if (lane == 0) {
                    cv[wid * kAdd + r] = x.v;
                    ci[wid * kAdd + r] = (double)x.i;
                }
                pv = x.v;
                pi = x.i;
            }
            if (lane == 0)
                for (; r < kAdd; ++r) {
                    cv[wid * kAdd + r] = -1.0;
                    ci[wid * kAdd + r] = -1.0;
                }
            __syncthreads();
            if (wid == 0) {
                double mv[2];
                int mi[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    mv[e] = cv[lane + 64 * e];
                    mi[e] = (int)ci[lane + 64 * e];
                }
                pv = INFINITY;
                pi = -1;
                int n = 0;
                for (; n < kmax; ++n) {
                    VI x; x.v = -1.0; x.i = -1;
#pragma unroll
                    for (int e = 0; e < 2; ++e)
                        if (mi[e] >= 0 && (mv[e] < pv || (mv[e] == pv && mi[e] > pi))) {
                            VI cc; cc.v = mv[e]; cc.i = mi[e];
                            x = vmax(x, cc);
                        }
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        VI y;
                        y.v = __shfl_xor(x.v, o, 64);
                        y.i = __shfl_xor(x.i, o, 64);
                        x = vmax(x, y);
                    }
                    if (x.i < 0) break;
                    if (lane == 0) {
                        list[n] = x.i;
                        v.th[x.i] = (signed char)sgn(v.g[x.i]);
                    }
                    pv = x.v;
                    pi = x.i;
                }
                if (lane == 0) red.count = n;
            }
            __syncthreads();
            nadd = red.count;
            __syncthreads();
        }
        SUB(18);
        if (nadd > 0) {
#ifdef PAM_PHASE_PROFILE
            n_add += nadd;
#endif
            if (!activate(v, list, nadd, red, cinv, blk, tile, zv && !ex)) {
                // none could enter: rebuild the block inverse (at most twice
                // per phase) and take the step again from the same point
                if (rebuilds >= 2) break;
                ++rebuilds;
                rebuild(v, list, red, cinv, blk, tile);
                zv = false;
                n_inc = 0;
                skip_solve = false;
                continue;
            }
            n_inc += 1;
            refines = 0;
#ifdef PAM_INC_CHECK
            dbg_op = 3;
#endif
            PHASE_MARK(7);
            continue;
        }
        if (v.pend > 0) {
            // a staged frozen set and nothing to activate: apply it, then
            // select again with its coordinates inactive
            flush_pending(v, tile);
            skip_solve = true;
            continue;
        }
        // optimal up to the reduced-system residual r_S = g_S - lambda1 theta_S
        const int s = v.s;
        double rp = 0.0;
        for (int i = threadIdx.x; i < s; i += kT) {
            const int k = v.S[i];
            v.rhs[i] = v.g[k] - v.l1 * (double)v.th[k];
            rp = fmax(rp, fabs(v.rhs[i]));
        }
        const double rmax = bmax(rp, red);
        if (s == 0 || rmax <= gtol || refines >= 3) {
            status = PAM_ST_OK;
            break;
        }
        ++refines;
        zv = false;
        if (ex) continue;   // the next CG solve starts from beta: a refinement step
        solve_active(v, v.rhs, v.z, red);   // correction H r
        bool keep_mine = true;
        for (int i = threadIdx.x; i < s; i += kT) {
            const int k = v.S[i];
            if ((int)sgn(v.beta[k] + v.z[i]) != v.th[k]) keep_mine = false;
        }
        if (ball(keep_mine, red)) {
            for (int i = threadIdx.x; i < s; i += kT) v.beta[v.S[i]] += v.z[i];
            __syncthreads();
            skip_solve = true;
        }
    }
    }   // phase
    // ---- outputs and KKT residual
    __syncthreads();
    if constexpr (kLow) {
        if (!ran_ex) full_gradient(v);
        else if (status != PAM_ST_OK) grad64(v, P);
    } else {
        full_gradient(v);
    }
    double kk = 0.0, nz = 0.0;
    for (int m = threadIdx.x; m < M; m += kT) {
        const double b = v.beta[m];
        const double e = b != 0.0 ? fabs(v.g[m] - v.l1 * sgn(b)) : fmax(fabs(v.g[m]) - v.l1, 0.0);
        kk = fmax(kk, e);
        nz += b != 0.0 ? 1.0 : 0.0;
    }
    const double kkt = bmax(kk, red);
#ifdef PAM_INC_CHECK
    if (kkt > 1e-8)
        for (int m = threadIdx.x; m < M; m += kT) {
            const double b = v.beta[m];
            const double e = b != 0.0 ? fabs(v.g[m] - v.l1 * sgn(b)) : fmax(fabs(v.g[m]) - v.l1, 0.0);
            if (e > 1e-8)
                printf("KKT sub=%d m=%d beta=%.3e g=%.3e th=%d pos=%d status=%d it=%d refines=%d\n", s_id, m, b, v.g[m],
                       (int)v.th[m], v.pos[m], status, it, refines);
        }
#endif
    const double nzs = bsum(nz, red);
    for (int m = threadIdx.x; m < a.m_cap; m += kT) beta_out[m] = m < M ? v.beta[m] : 0.0;
#ifdef PAM_PHASE_PROFILE
    if (threadIdx.x == 0 && s_id < kPhaseSubs) {
        double *o = g_phase + (size_t)s_id * kPhaseW;
        for (int k = 0; k < 8; ++k) { o[k] = ph[k] * 0.01; o[8 + k] = phb[k]; }
        o[16] = M; o[17] = s_init; o[18] = v.s; o[19] = it; o[20] = n_cons; o[21] = n_ls; o[22] = n_rm;
        o[23] = n_add; o[24] = sweeps; o[25] = ran_ex ? it - it_ex0 : 0; o[26] = n_cg;
        o[27] = ran_ex ? (wall_clock64() - t_ex0) * 0.01 : 0.0;
        o[28] = 0.01 * (double)(wall_clock64() - t_begin);
        o[29] = 1.0;
        for (int k = 0; k < 23; ++k) o[30 + k] = 0.01 * (double)v.sp[k];
    }
#endif
    if (v.tsh[3]) status = PAM_ST_NOCONV;   // a team member did not answer: the result is not certified
    if (st && threadIdx.x == 0) {
        st->status = status;
        st->cd_sweeps = sweeps;
        st->iters = it;
        st->support = (int)nzs;
        st->kkt = kkt;
        st->stream_bytes = v.bytes;
        st->polish = n_cg;
        st->team = v.T;
        st->solve_us = 0.01 * (double)(wall_clock64() - t_begin);
    }
}

// LDS of one workgroup on gfx950 (static + dynamic)

// Entry points of the kernel instances, one translation unit per group (the
// instances compile in parallel): the LDS-vector instances of one Gram type
// (team = with team code), and the HBM-vector instances of both types.
const void *solve_kernel_f64(bool team);
const void *solve_kernel_f32(bool team);
const void *solve_kernel_vg(bool f64);
#ifdef PAM_PHASE_PROFILE
// phase records of the profile build (each unit holds its own buffer):
// clear (host == nullptr) or read kPhaseSubs * kPhaseW doubles
hipError_t solve_phase_io_f64(double *host, hipStream_t st);
hipError_t solve_phase_io_f32(double *host, hipStream_t st);
hipError_t solve_phase_io_vg(double *host, hipStream_t st);
#endif

}  // namespace pam
