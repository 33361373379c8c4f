// Solve kernel instances: vg (iteration vectors in HBM, both Gram types).
#include "k_solve_impl.h"

namespace pam {

const void *solve_kernel_vg(bool f64) {
    return f64 ? (const void *)k_solve<double, false, true> : (const void *)k_solve<float, false, true>;
}

#ifdef PAM_PHASE_PROFILE
hipError_t solve_phase_io_vg(double *host, hipStream_t st) {
    const size_t bytes = (size_t)kPhaseSubs * kPhaseW * sizeof(double);
    if (!host) {
        std::vector<double> z((size_t)kPhaseSubs * kPhaseW, 0.0);
        hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_phase), z.data(), bytes, 0, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    }
    hipError_t e = hipMemcpyFromSymbolAsync(host, HIP_SYMBOL(g_phase), bytes, 0, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}
#endif

}  // namespace pam
