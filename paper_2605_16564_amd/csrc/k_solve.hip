// Host side of the elastic-net solve: capacity and LDS sizing, team size,
// and the launch (the kernel and its instances: k_solve_impl.h and the
// k_solve_*.hip units).
#include "k_solve_impl.h"

namespace pam {

__host__ __device__ size_t solve_ldh(int m_cap) { return ldh_of(m_cap); }
__host__ __device__ size_t solve_h_elems(int m_cap) { return h_elems_of(m_cap); }
__host__ __device__ size_t solve_scratch_elems(int m_cap, int npad, int precision, int team, bool vg) {
    return scratch_elems_of(m_cap, npad, precision, team, vg);
}
size_t solve_lds_bytes(int m_cap) { return (size_t)57 * round_up(m_cap, 8) + 64; }   // 57 B per center: see the carve-out in k_solve

static constexpr size_t kLdsPerWorkgroup = 160 * 1024;
static constexpr int kSolveMaxCap = 32768;   // H alone is then 8.6 GB per subdomain

template <typename TG>
static const void *solve_fn(bool team) {
    return sizeof(TG) == sizeof(double) ? solve_kernel_f64(team) : solve_kernel_f32(team);
}

template <typename TG>
static const void *solve_fn_vg() { return solve_kernel_vg(sizeof(TG) == sizeof(double)); }

// Largest dictionary capacity whose per-center vectors fit LDS beside the
// static LDS of the (team) instance; beyond it the vectors go to HBM.
static int lds_capacity(int precision) {
    static int cap[2] = {-1, -1};
    const int k = precision == PAM_PREC_F64 ? 0 : 1;
    if (cap[k] < 0) {
        hipFuncAttributes attr;   // the team instance's static LDS includes the other's
        const void *fn = precision == PAM_PREC_F64 ? solve_fn<double>(true) : solve_fn<float>(true);
        if (hipFuncGetAttributes(&attr, fn) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        cap[k] = (int)(((kLdsPerWorkgroup - attr.sharedSizeBytes - 64) / 57) / 8 * 8);
    }
    return cap[k];
}

bool solve_vectors_global(int m_cap, int precision) { return m_cap > lds_capacity(precision); }

pam_status solve_check_capacity(int m_cap, int precision) {
    (void)precision;
    if (m_cap > kSolveMaxCap) {
        char msg[160];
        snprintf(msg, sizeof msg, "m_cap too large for the solve (%d; max %d)", m_cap, kSolveMaxCap);
        set_error(msg);
        return PAM_ERR_CAPACITY;
    }
    return PAM_OK;
}

// The dynamic-LDS limit of both instances of one Gram type, set only when it
// changes (so that launches inside a graph capture make no attribute calls
// once the size is settled).
template <typename TG>
static pam_status solve_set_lds(size_t lds) {
    static size_t current = 0;
    if (current == lds) return PAM_OK;
    for (bool team : {false, true})
        PAM_CHECK_HIP(hipFuncSetAttribute(solve_fn<TG>(team), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    current = lds;
    return PAM_OK;
}

pam_status solve_prepare(int m_cap, int precision) {
    if (solve_vectors_global(m_cap, precision)) return PAM_OK;   // no dynamic LDS
    const size_t lds = solve_lds_bytes(m_cap);
    return precision == PAM_PREC_F64 ? solve_set_lds<double>(lds) : solve_set_lds<float>(lds);
}

size_t solve_team_ctl_bytes(int sub_count) { return (size_t)sub_count * kCtl * sizeof(unsigned long long); }

int solve_team_size(int sub_count, int m_cap, int precision, int requested) {
    if (requested == 1 || sub_count < 1 || solve_vectors_global(m_cap, precision)) return 1;
    const size_t lds = solve_lds_bytes(m_cap);
    const void *fn = precision == PAM_PREC_F64 ? solve_fn<double>(true) : solve_fn<float>(true);
    if ((precision == PAM_PREC_F64 ? solve_set_lds<double>(lds) : solve_set_lds<float>(lds)) != PAM_OK) return 1;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kT, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    const long long resident = (long long)per_cu * cus;
    int T = requested >= 2 ? std::min(requested, kTeamMax) : kTeamMax;
    while (T > 1 && round_up(sub_count, 8) * T > resident) T /= 2;
    return T;
}

pam_status launch_solve(pam_ctx *ctx, const FitArgs &a) {
    const size_t lds = solve_lds_bytes(a.m_cap);
    pam_status st = solve_check_capacity(a.m_cap, a.precision);
    if (st != PAM_OK) return st;
    double *H = wsp<double>(ctx, BUF_H);
    double *scr = wsp<double>(ctx, BUF_VEC);
    const int32_t *flags = wsp<int32_t>(ctx, BUF_FLAGS);
    const int T = a.team > 1 ? a.team : 1;
    unsigned long long *tctl = nullptr;
    if (T > 1) {
        // control words start at zero (no command posted) for every launch
        const size_t bytes = solve_team_ctl_bytes(a.sub_count);
        if ((st = ensure(ctx, BUF_TEAM, bytes)) != PAM_OK) return st;
        tctl = wsp<unsigned long long>(ctx, BUF_TEAM);
        if ((st = launch_fill_u32(ctx, tctl, 0u, (int64_t)(bytes / 4))) != PAM_OK) return st;
    }
    const bool f64 = a.precision == PAM_PREC_F64;
    const bool vg = solve_vectors_global(a.m_cap, a.precision);
    if (!vg && (st = f64 ? solve_set_lds<double>(lds) : solve_set_lds<float>(lds)) != PAM_OK) return st;
    const void *fn = vg ? (f64 ? solve_fn_vg<double>() : solve_fn_vg<float>())
                        : (f64 ? solve_fn<double>(T > 1) : solve_fn<float>(T > 1));
    FitArgs ka = a;
    void *G = f64 ? (void *)wsp<double>(ctx, BUF_G) : (void *)wsp<float>(ctx, BUF_G);
    void *args[] = {&ka, &G, &H, &scr, (void *)&flags, &tctl};
    // A team grid is no larger than what the device holds at once
    // (solve_team_size), so its workgroups run together on an idle device; an
    // ordinary launch suffices because no wait depends on residency to end.
    const unsigned blocks = T > 1 ? (unsigned)(round_up(a.sub_count, 8) * T) : (unsigned)a.sub_count;
#ifdef PAM_PHASE_PROFILE
    auto phase_io = vg ? solve_phase_io_vg : f64 ? solve_phase_io_f64 : solve_phase_io_f32;
    PAM_CHECK_HIP(phase_io(nullptr, ctx->stream));
#endif
    PAM_CHECK_HIP(hipLaunchKernel(fn, dim3(blocks), dim3(kT), args, vg ? 0 : lds, ctx->stream));
    PAM_CHECK_HIP(hipGetLastError());
#ifdef PAM_PHASE_PROFILE
    {
        std::vector<double> o((size_t)kPhaseSubs * kPhaseW);
        PAM_CHECK_HIP(phase_io(o.data(), ctx->stream));
        for (int sidx = a.sub_begin; sidx < a.sub_begin + a.sub_count && sidx < kPhaseSubs; ++sidx) {
            const double *r = &o[(size_t)sidx * kPhaseW];
            if (r[29] != 1.0) continue;
            printf("PH sub=%d M=%.0f s_init=%.0f s=%.0f it=%.0f cons=%.0f ls=%.0f rm=%.0f add=%.0f sweeps=%.0f it_ex=%.0f "
                   "cg=%.0f us: grad0=%.0f cd=%.0f init=%.0f solve=%.0f ls=%.0f rm=%.0f fullg=%.0f act=%.0f ex=%.0f "
                   "total=%.0f\n", sidx, r[16], r[17], r[18], r[19], r[20], r[21], r[22], r[23], r[24], r[25], r[26],
                   r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[27], r[28]);
            printf("SP sub=%d us: gather=%.0f upass=%.0f pendfix=%.0f cmat=%.0f chol=%.0f vmat=%.0f updz=%.0f "
                   "hupd=%.0f border=%.0f freeze=%.0f cpv=%.0f cphupd=%.0f cpdrop=%.0f grad=%.0f hgemv=%.0f lsupd=%.0f "
                   "inc=%.0f fzscan=%.0f select=%.0f cg=%.0f w64=%.0f grad64=%.0f excompact=%.0f\n", sidx,
                   r[30], r[31], r[32], r[33], r[34], r[35], r[36], r[37], r[38], r[39], r[40], r[41], r[42], r[43],
                   r[44], r[45], r[46], r[47], r[48], r[49], r[50], r[51], r[52]);
            printf("PB sub=%d MB: grad0=%.1f cd=%.1f init=%.1f solve=%.1f ls=%.1f rm=%.1f fullg=%.1f act=%.1f\n", sidx,
                   r[8] * 1e-6, r[9] * 1e-6, r[10] * 1e-6, r[11] * 1e-6, r[12] * 1e-6, r[13] * 1e-6, r[14] * 1e-6,
                   r[15] * 1e-6);
        }
        fflush(stdout);
    }
#endif
    return PAM_OK;
}

}  // namespace pam
