// Launch entry points of the kernel files, called by the host runtime.
#pragma once

#include "lcf_internal.h"

namespace lcf {

struct RuleParams {
    int cut, shape, pd_mode, k_fixed;
    double beta_knee, knee_max_frac, beta_sigmoid, beta_median, slope_thr, beta_power;
};

hipError_t launch_windows(const Workspace& ws, hipStream_t st);
hipError_t launch_gram(const Workspace& ws, bool defl, bool reduce, int precision, hipStream_t st);
int gram_tiles(int ntp, bool defl);
hipError_t launch_tissue(const Workspace& ws, double rho, int iters, hipStream_t st);
hipError_t launch_assemble(const Workspace& ws, int keep_r, hipStream_t st);
hipError_t launch_evd(const Workspace& ws, int max_sweeps, int nt_max, int method, hipStream_t st);
hipError_t launch_evd_vectors(const Workspace& ws, int method, int all, int max_sweeps, int nt_max, hipStream_t st);
hipError_t launch_heevd(int n, int nt, const double2* a, double* w, double2* v, int* sweeps,
                        double2* work, int max_sweeps, int* flags, hipStream_t st);
hipError_t launch_rules(const Workspace& ws, const RuleParams& rp, hipStream_t st);
// Sliding packets: R_new from R_old shifted by `hop` frames plus the hop new
// columns in FP64 (part: stream_partial_elems(S, ntp) double2), then R_new as
// the FP32 pass-1 covariance and the pass-2 Gram of the assembly.
hipError_t launch_cov_stream(const Workspace& ws, const double2* rold, double2* rnew, double2* part, int hop,
                             hipStream_t st);
size_t stream_partial_elems(int S, int ntp);
// Method 4 (Eq. 8): V / sigma in the original basis, then the per-chunk sums of
// the NCC curve (partials, added by the rules kernel). Needs every eigenvector.
hipError_t launch_ncc(const Workspace& ws, hipStream_t st);
hipError_t launch_projector(const Workspace& ws, int precision, hipStream_t st);
hipError_t launch_reproj(const Workspace& ws, int precision, hipStream_t st);
hipError_t launch_export(const Workspace& ws, int first, int count, int nt, double* eigvals, float* weights,
                         int* k, int* sweeps, int* flags, double* alpha, int* rank, double2* eigvecs,
                         double* curve, double* mlp_gate, hipStream_t st);
hipError_t launch_export_cov(const Workspace& ws, int first, int count, int nt, double2* cov, hipStream_t st);
hipError_t launch_flags_or(const Workspace& ws, int* sticky, hipStream_t st);

// ---- learned weights (k_mlp.hip)
constexpr int MLP_NT = 128;
constexpr int MLP_H = 256;
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_NT;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_NT * MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B3 + MLP_NT;   // 131712

struct MlpDev {
    float* master;   // FP32 parameters
    uint16_t* wbf;   // BF16 working copy (same layout)
    float* m;        // Adam moments
    float* v;
    float* grad;     // last gradients
};

hipError_t mlp_forward(const MlpDev& net, const float* z, int rows, float* scratch, float* wout, hipStream_t st);
hipError_t mlp_features(const double* lam, int ldl, int rows, float* z, int* valid, hipStream_t st);
// gate_db < 0: no gate; gate_out (may be null): [S] predicted deviation (dB)
hipError_t mlp_apply(const Workspace& ws, const float* wout, const int* valid, int pd_mode, double gate_db,
                     double* gate_out, hipStream_t st);
hipError_t mlp_refresh_bf16(const MlpDev& net, hipStream_t st);
hipError_t mlp_train_step(const MlpDev& net, const double* lam, const float* target, int rows, float lr, int step,
                          float* scratch, float* loss_out, hipStream_t st);
size_t mlp_train_scratch_floats(int rows);
size_t mlp_infer_scratch_floats(int rows);

}  // namespace lcf
