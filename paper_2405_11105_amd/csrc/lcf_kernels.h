// Launch entry points of the kernel files, called by the host runtime.
#pragma once

#include "lcf_internal.h"

namespace lcf {

struct RuleParams {
    int cut, shape, pd_mode, k_fixed;
    double beta_knee, knee_max_frac, beta_sigmoid;
};

hipError_t launch_windows(const Workspace& ws, hipStream_t st);
hipError_t launch_gram(const Workspace& ws, bool defl, bool reduce, int precision, hipStream_t st);
int gram_tiles(int ntp, bool defl);
hipError_t launch_tissue(const Workspace& ws, double rho, int iters, hipStream_t st);
hipError_t launch_assemble(const Workspace& ws, hipStream_t st);
hipError_t launch_jacobi(const Workspace& ws, int max_sweeps, int nt_max, hipStream_t st);
hipError_t launch_heevd(int n, int nt, const double2* a, double* w, double2* v, int* sweeps,
                        double2* work, int max_sweeps, int* flags, hipStream_t st);
hipError_t launch_rules(const Workspace& ws, const RuleParams& rp, hipStream_t st);
hipError_t launch_projector(const Workspace& ws, int precision, hipStream_t st);
hipError_t launch_reproj(const Workspace& ws, int precision, hipStream_t st);
hipError_t launch_export(const Workspace& ws, int first, int count, int nt, double* eigvals, float* weights,
                         int* k, int* sweeps, int* flags, double* alpha, int* rank, double2* eigvecs,
                         hipStream_t st);
hipError_t launch_export_cov(const Workspace& ws, int first, int count, int nt, double2* cov, hipStream_t st);
hipError_t launch_flags_or(const Workspace& ws, int* sticky, hipStream_t st);

}  // namespace lcf
