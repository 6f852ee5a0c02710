// Learned eigencomponent weights: a 128-256-256-128 MLP (GELU, GELU, sigmoid)
// from the normalised log-eigenvalue spectrum of a subset to soft weights for
// the projection of Eq. 4 (the role of the rules of Eqs 6 and 9).
//
// Weights are BF16 working copies of an FP32 master; activations and deltas are
// FP32 in HBM and split into BF16 hi + lo on load, so each GEMM is 2 (forward,
// dX) or 3 (dW) MFMA products per tile with FP32 accumulation.
#include <math.h>

#include "lcf_internal.h"
#include "lcf_kernels.h"

namespace lcf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t mlp_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float gelu_f(float h) { return 0.5f * h * (1.0f + erff(h * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float h) {
    return 0.5f * (1.0f + erff(h * 0.70710678118654752f)) + h * expf(-0.5f * h * h) * 0.3989422804014327f;
}

constexpr int GK = 32;     // K step (one BF16 MFMA)
constexpr int GLD = GK + 8;

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS_SIGMOID = 2, EPI_GELU_GRAD = 3 };

// C[m][n] = sum_k A(m,k) B(k,n) with A(m,k) = a[m*sam + k*sak] (FP32, split
// hi/lo when asplit) and B(k,n) = b[k*sbk + n*sbn]; B is BF16 (weights, bw != 0)
// or FP32 split hi/lo. Epilogues: store; +bias, keep pre-activation in aux and
// GELU in c; +bias then sigmoid; multiply by GELU'(aux).
struct GemmArgs {
    const float* a;
    long sam, sak;
    const float* bf;            // FP32 B (or null)
    const uint16_t* bw;         // BF16 B (or null)
    long sbk, sbn;
    float* c;
    long ldc;
    float* aux;                 // pre-activation store (EPI_BIAS_GELU) or GELU input (EPI_GELU_GRAD)
    const float* bias;
    int M, N, K;
    int asplit, bsplit;
};

// GT x GT output tiles (64, or 32 for the small products of inference so that
// more work-groups share the chip), four waves in a 2 x 2 layout.
template <int EPI, int GT>
__global__ void __launch_bounds__(256) k_mlp_gemm(GemmArgs g) {
    constexpr int WT = GT / 32;            // 16 x 16 blocks per wave and axis
    __shared__ __attribute__((aligned(16))) uint16_t Ah[GT * GLD], Al[GT * GLD], Bh[GT * GLD], Bl[GT * GLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gq = lane >> 4, col = lane & 15;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wy = wave >> 1, wx = wave & 1;
    floatx4 acc[WT][WT];
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        __syncthreads();
        for (int e = tid; e < GT * GK; e += 256) {
            int m, k;
            if (g.sak == 1) { m = e / GK; k = e % GK; } else { m = e % GT; k = e / GT; }
            float v = 0.f;
            if (m0 + m < g.M && k0 + k < g.K) v = g.a[(long)(m0 + m) * g.sam + (long)(k0 + k) * g.sak];
            const uint32_t h = mlp_bf16(v);
            Ah[m * GLD + k] = (uint16_t)h;
            Al[m * GLD + k] = (uint16_t)mlp_bf16(v - __uint_as_float(h << 16));
        }
        for (int e = tid; e < GT * GK; e += 256) {
            int n, k;
            if (g.sbk == 1) { n = e / GK; k = e % GK; } else { n = e % GT; k = e / GT; }
            uint16_t hb = 0, lb = 0;
            if (n0 + n < g.N && k0 + k < g.K) {
                const long off = (long)(k0 + k) * g.sbk + (long)(n0 + n) * g.sbn;
                if (g.bw) hb = g.bw[off];
                else {
                    const float v = g.bf[off];
                    const uint32_t h = mlp_bf16(v);
                    hb = (uint16_t)h;
                    lb = (uint16_t)mlp_bf16(v - __uint_as_float(h << 16));
                }
            }
            Bh[n * GLD + k] = hb;
            Bl[n * GLD + k] = lb;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < WT; ++i) {
            const int mr = wy * 16 * WT + i * 16 + col;
            const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(Ah + mr * GLD + 8 * gq));
            const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(Al + mr * GLD + 8 * gq));
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                const int nr = wx * 16 * WT + j * 16 + col;
                const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(Bh + nr * GLD + 8 * gq));
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[i][j], 0, 0, 0);
                if (g.asplit) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[i][j], 0, 0, 0);
                if (g.bsplit) {
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(Bl + nr * GLD + 8 * gq));
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[i][j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wy * 16 * WT + i * 16 + 4 * gq + r;
                const int n = n0 + wx * 16 * WT + j * 16 + col;
                if (m >= g.M || n >= g.N) continue;
                const long o = (long)m * g.ldc + n;
                float v = acc[i][j][r];
                if (EPI == EPI_BIAS_GELU) {
                    v += g.bias[n];
                    g.aux[o] = v;
                    g.c[o] = gelu_f(v);
                } else if (EPI == EPI_BIAS_SIGMOID) {
                    v += g.bias[n];
                    g.c[o] = 1.0f / (1.0f + expf(-v));
                } else if (EPI == EPI_GELU_GRAD) {
                    g.c[o] = v * gelu_grad_f(g.aux[o]);
                } else {
                    g.c[o] = v;
                }
            }
}

template <int EPI>
static hipError_t gemm(const GemmArgs& g, hipStream_t st) {
    // 64 x 64 tiles while they give at least one work-group per CU (training),
    // 32 x 32 below (inference over the subsets of a call)
    const long tiles64 = (long)((g.N + 63) / 64) * ((g.M + 63) / 64);
    if (tiles64 >= 256) {
        const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
        hipLaunchKernelGGL((k_mlp_gemm<EPI, 64>), grid, dim3(256), 0, st, g);
    } else {
        const dim3 grid((g.N + 31) / 32, (g.M + 31) / 32);
        hipLaunchKernelGGL((k_mlp_gemm<EPI, 32>), grid, dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

// Features z = log10(max(lambda, lambda_1 2^-52) / lambda_1) / 8 from FP64
// eigenvalues (row stride ldl); rows with lambda_1 <= 0 or non-finite values
// are marked invalid (the caller keeps the rule weights there).
__global__ void __launch_bounds__(128) k_mlp_features(const double* lam, int ldl, int rows, float* z, int* valid) {
    const int b = blockIdx.x, i = threadIdx.x;
    if (b >= rows) return;
    const double l1 = lam[(long)b * ldl];
    const double li = lam[(long)b * ldl + i];
    const bool ok = l1 > 0.0 && isfinite(l1) && isfinite(li);
    const double l = li > l1 * 2.220446049250313e-16 ? li : l1 * 2.220446049250313e-16;
    z[(long)b * MLP_NT + i] = ok ? (float)(log10(l / l1) * 0.125) : 0.f;
    const int bad = __syncthreads_or(!ok);
    if (i == 0 && valid) valid[b] = !bad;
}

// Loss sum_i c_i (w_i - t_i)^2 and d(loss)/dh3 = 2 c (w - t) w (1 - w) / B with
// c_i = lambda_i / sum_j lambda_j t_j^2; one block per row, then a fixed-order sum.
__global__ void __launch_bounds__(128) k_mlp_loss_rows(const double* lam, const float* w, const float* t, int rows,
                                                       float* d3, double* row_loss) {
    __shared__ double red[2];
    const int b = blockIdx.x, i = threadIdx.x;
    const long o = (long)b * MLP_NT + i;
    const double tt = (double)t[o];
    double e = wave_sum(lam[o] * tt * tt);
    if ((i & 63) == 0) red[i >> 6] = e;
    __syncthreads();
    const double en = red[0] + red[1] > 0.0 ? red[0] + red[1] : 1.0;
    const double c = lam[o] / en;
    const double diff = (double)w[o] - tt;
    d3[o] = (float)(2.0 * c * diff * (double)w[o] * (1.0 - (double)w[o]) / rows);
    double l = wave_sum(c * diff * diff);
    __syncthreads();
    if ((i & 63) == 0) red[i >> 6] = l;
    __syncthreads();
    if (i == 0) row_loss[b] = red[0] + red[1];
}

__global__ void __launch_bounds__(64) k_mlp_loss_sum(const double* row_loss, int rows, float* loss_out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < rows; ++b) s += row_loss[b];
    if (loss_out) *loss_out = (float)(s / rows);
}

// Column sums (bias gradients) in fixed order.
__global__ void __launch_bounds__(256) k_mlp_colsum(const float* d, int rows, int cols, float* out) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= cols) return;
    double s = 0.0;
    for (int b = 0; b < rows; ++b) s += d[(long)b * cols + n];
    out[n] = (float)s;
}

// Adam on the FP32 master, then refresh the BF16 working copy.
__global__ void __launch_bounds__(256) k_mlp_adam(float* master, uint16_t* wbf, float* m, float* v, const float* grad,
                                                  int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gr = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gr;
    const float vi = b2 * v[i] + (1.f - b2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    const float p = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    master[i] = p;
    wbf[i] = (uint16_t)mlp_bf16(p);
}

__global__ void __launch_bounds__(256) k_mlp_to_bf16(const float* master, uint16_t* wbf, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) wbf[i] = (uint16_t)mlp_bf16(master[i]);
}

// Replace the rule weights of valid subsets by the network output and
// recompute alpha_d (Eq. 13) with them; invalid subsets keep the rule and are
// flagged. With the gate on (gate_db >= 0), the rule is also kept (and the
// subset flagged) when the predicted power Doppler deviation of the network's
// weights from the rule's reaches gate_db. After Eq. 13 a subset's power
// Doppler at pixel x is Npix Nt sum_i q_i e_i(x), with q_i = w_i^2 lambda_i /
// sum_j w_j^2 lambda_j the component's share of the filtered energy and
// e_i(x) = |(C_w v_i)(x)|^2 / lambda_i the same for either weight set, so the
// ratio of the two images at any pixel lies between the extreme ratios
// q_i(net) / q_i(rule) of the components present there. The prediction is
// the largest |10 log10| of that ratio over components holding at least
// GATE_SHARE of either filtered energy (infinite when only one set keeps
// such a component, or when either energy is zero). gate_out[s * ntp] (may be
// null) receives it.
constexpr double GATE_SHARE = 1e-3;

__global__ void __launch_bounds__(128) k_mlp_apply(Workspace ws, const float* wout, const int* valid, int pd_mode,
                                                   double gate_db, double* gate_out) {
    __shared__ double red[4];
    const int s = blockIdx.x, i = threadIdx.x, ntp = ws.ntp;
    if (!valid || !valid[s] || ws.sub[s].nt != MLP_NT) {
        if (i == 0) {
            atomicOr(&ws.flags[s], 8);
            if (gate_out) gate_out[(long)s * ntp] = INFINITY;
        }
        return;
    }
    const double w = (double)wout[(long)s * MLP_NT + i];
    const double l = ws.lam[(long)s * ntp + i];
    const double wr = ws.wts[(long)s * ntp + i];
    const double em = w * w * l, er = wr * wr * l;
    const double sm = wave_sum(em), sr = wave_sum(er);
    if ((i & 63) == 0) { red[i >> 6] = sm; red[2 + (i >> 6)] = sr; }
    __syncthreads();
    const double en = red[0] + red[1], enr = red[2] + red[3];
    // predicted deviation (dB) of this component's share
    double g = 0.0;
    if (!(en > 0.0) || !(enr > 0.0)) {
        g = INFINITY;
    } else if (l > 0.0) {
        const double q = em / en, p = er / enr;
        if (q >= GATE_SHARE || p >= GATE_SHARE) g = (q > 0.0 && p > 0.0) ? fabs(10.0 * log10(q / p)) : INFINITY;
    }
    for (int m = 32; m >= 1; m >>= 1) g = fmax(g, __shfl_xor(g, m, 64));
    __syncthreads();
    if ((i & 63) == 0) red[i >> 6] = g;
    __syncthreads();
    const double gmax = fmax(red[0], red[1]);
    if (i == 0 && gate_out) gate_out[(long)s * ntp] = gmax;
    if (gate_db >= 0.0 && !(gmax < gate_db)) {
        if (i == 0) atomicOr(&ws.flags[s], 8);
        return;                                  // the rule's weights and alpha stay
    }
    ws.wts[(long)s * ntp + i] = w;
    if (i == 0) {
        ws.alpha[s] = pd_mode == 1 ? 1.0 : (en > 0.0 ? ws.sub[s].npix_nt / en : 0.0);
        ws.kcut[s] = -1;
    }
}

// ------------------------------------------------------------------ driver

// Forward of `rows` spectra: z [rows][128] -> w [rows][128]; scratch holds
// h1, a1, h2, a2 ([rows][256] each).
hipError_t mlp_forward(const MlpDev& net, const float* z, int rows, float* scratch, float* wout, hipStream_t st) {
    float* h1 = scratch;
    float* a1 = h1 + (long)rows * MLP_H;
    float* h2 = a1 + (long)rows * MLP_H;
    float* a2 = h2 + (long)rows * MLP_H;
    GemmArgs g{};
    g.a = z; g.sam = MLP_NT; g.sak = 1;
    g.bw = net.wbf + MLP_OFF_W1; g.sbk = 1; g.sbn = MLP_NT;
    g.c = a1; g.ldc = MLP_H; g.aux = h1; g.bias = net.master + MLP_OFF_B1;
    g.M = rows; g.N = MLP_H; g.K = MLP_NT; g.asplit = 1; g.bsplit = 0;
    hipError_t e = gemm<EPI_BIAS_GELU>(g, st);
    if (e != hipSuccess) return e;
    g.a = a1; g.sam = MLP_H;
    g.bw = net.wbf + MLP_OFF_W2; g.sbn = MLP_H;
    g.c = a2; g.aux = h2; g.bias = net.master + MLP_OFF_B2; g.K = MLP_H;
    e = gemm<EPI_BIAS_GELU>(g, st);
    if (e != hipSuccess) return e;
    g.a = a2; g.bw = net.wbf + MLP_OFF_W3; g.sbn = MLP_H;
    g.c = wout; g.ldc = MLP_NT; g.aux = nullptr; g.bias = net.master + MLP_OFF_B3; g.N = MLP_NT;
    return gemm<EPI_BIAS_SIGMOID>(g, st);
}

hipError_t mlp_features(const double* lam, int ldl, int rows, float* z, int* valid, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_features, dim3(rows), dim3(MLP_NT), 0, st, lam, ldl, rows, z, valid);
    return hipGetLastError();
}

hipError_t mlp_apply(const Workspace& ws, const float* wout, const int* valid, int pd_mode, double gate_db,
                     double* gate_out, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_apply, dim3(ws.S), dim3(MLP_NT), 0, st, ws, wout, valid, pd_mode, gate_db, gate_out);
    return hipGetLastError();
}

hipError_t mlp_refresh_bf16(const MlpDev& net, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, net.master, net.wbf,
                       MLP_NPARAM);
    return hipGetLastError();
}

// One training step on `rows` spectra (lam FP64 [rows][128], target FP32).
hipError_t mlp_train_step(const MlpDev& net, const double* lam, const float* target, int rows, float lr, int step,
                          float* scratch, float* loss_out, hipStream_t st) {
    float* z = scratch;
    float* h1 = z + (long)rows * MLP_NT;
    float* a1 = h1 + (long)rows * MLP_H;
    float* h2 = a1 + (long)rows * MLP_H;
    float* a2 = h2 + (long)rows * MLP_H;
    float* w = a2 + (long)rows * MLP_H;
    float* d3 = w + (long)rows * MLP_NT;
    float* d2 = d3 + (long)rows * MLP_NT;
    float* d1 = d2 + (long)rows * MLP_H;
    double* rl = reinterpret_cast<double*>(d1 + (long)rows * MLP_H);
    hipError_t e = mlp_features(lam, MLP_NT, rows, z, nullptr, st);
    if (e != hipSuccess) return e;
    e = mlp_forward(net, z, rows, h1, w, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_loss_rows, dim3(rows), dim3(MLP_NT), 0, st, lam, w, target, rows, d3, rl);
    hipLaunchKernelGGL(k_mlp_loss_sum, dim3(1), dim3(64), 0, st, rl, rows, loss_out);
    float* gW1 = net.grad + MLP_OFF_W1;
    float* gW2 = net.grad + MLP_OFF_W2;
    float* gW3 = net.grad + MLP_OFF_W3;
    GemmArgs g{};
    // dW3 = d3^T a2  (M = 128, N = 256, K = rows)
    g.a = d3; g.sam = 1; g.sak = MLP_NT;
    g.bf = a2; g.sbk = MLP_H; g.sbn = 1;
    g.c = gW3; g.ldc = MLP_H; g.M = MLP_NT; g.N = MLP_H; g.K = rows; g.asplit = 1; g.bsplit = 1;
    if ((e = gemm<EPI_STORE>(g, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3(1), dim3(256), 0, st, d3, rows, MLP_NT, net.grad + MLP_OFF_B3);
    // d2 = (d3 W3) * GELU'(h2)  (M = rows, N = 256, K = 128); B(k,n) = W3[k][n]
    g = GemmArgs{};
    g.a = d3; g.sam = MLP_NT; g.sak = 1;
    g.bw = net.wbf + MLP_OFF_W3; g.sbk = MLP_H; g.sbn = 1;
    g.c = d2; g.ldc = MLP_H; g.aux = h2; g.M = rows; g.N = MLP_H; g.K = MLP_NT; g.asplit = 1;
    if ((e = gemm<EPI_GELU_GRAD>(g, st)) != hipSuccess) return e;
    // dW2 = d2^T a1
    g = GemmArgs{};
    g.a = d2; g.sam = 1; g.sak = MLP_H;
    g.bf = a1; g.sbk = MLP_H; g.sbn = 1;
    g.c = gW2; g.ldc = MLP_H; g.M = MLP_H; g.N = MLP_H; g.K = rows; g.asplit = 1; g.bsplit = 1;
    if ((e = gemm<EPI_STORE>(g, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3(1), dim3(256), 0, st, d2, rows, MLP_H, net.grad + MLP_OFF_B2);
    // d1 = (d2 W2) * GELU'(h1)
    g = GemmArgs{};
    g.a = d2; g.sam = MLP_H; g.sak = 1;
    g.bw = net.wbf + MLP_OFF_W2; g.sbk = MLP_H; g.sbn = 1;
    g.c = d1; g.ldc = MLP_H; g.aux = h1; g.M = rows; g.N = MLP_H; g.K = MLP_H; g.asplit = 1;
    if ((e = gemm<EPI_GELU_GRAD>(g, st)) != hipSuccess) return e;
    // dW1 = d1^T z
    g = GemmArgs{};
    g.a = d1; g.sam = 1; g.sak = MLP_H;
    g.bf = z; g.sbk = MLP_NT; g.sbn = 1;
    g.c = gW1; g.ldc = MLP_NT; g.M = MLP_H; g.N = MLP_NT; g.K = rows; g.asplit = 1; g.bsplit = 1;
    if ((e = gemm<EPI_STORE>(g, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3(1), dim3(256), 0, st, d1, rows, MLP_H, net.grad + MLP_OFF_B1);
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, net.master, net.wbf, net.m,
                       net.v, net.grad, MLP_NPARAM, lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

size_t mlp_train_scratch_floats(int rows) { return (size_t)rows * (3 * MLP_NT + 6 * MLP_H + 2); }
size_t mlp_infer_scratch_floats(int rows) { return (size_t)rows * (2 * MLP_NT + 4 * MLP_H); }

}  // namespace lcf
