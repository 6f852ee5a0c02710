/*
 * lcf.h -- C ABI of the localized EVD clutter filter for AMD MI355X (gfx950).
 *
 * Method: Huang et al., "Real-time Adaptive and Localized Spatiotemporal Clutter
 * Filtering for Ultrasound Small Vessel Imaging" (arXiv 2405.11105).
 *
 * The library takes one or more complex IQ packets S (Ny x Nx x Nt), a grid of
 * 2-D Gaussian spatial windows and a thresholding rule, and returns the clutter
 * filtered IQ and the recombined power Doppler image:
 *
 *   C      Casorati matrix of S, rows = pixels, columns = frames (Fig. 1)
 *   C_w    = W_d C, one Gaussian window per subset d               (Eq. 11)
 *   R_d    = C_w^H C_w                                              (Eqs 1, 12)
 *   R_d    = V Lambda V^H, eigenvalues descending                   (Eq. 2)
 *   w_i    eigencomponent weights: hard cut (Eq. 4), curvature rule (Eq. 6),
 *          median rule (Eq. 7), slope rule, normalised cross-correlation of
 *          tissue and blood images (Eq. 8), sigmoid (Eq. 9), eigenvalue power
 *          weighting (Eq. 10), caller-given, or a learned MLP
 *   Chat_d = C_w V diag(w) V^H                                      (Eqs 4, 5)
 *   PD_d   = sum_t |Chat_d|^2                                       (text after Eq. 5)
 *   PD     = sum_d alpha_d PD_d, alpha_d = 1 / mean flow power      (Eq. 13)
 *
 * Conventions shared by every entry point:
 *  - Packets are complex64 (interleaved float re, im), C-contiguous [nt][ny][nx]:
 *    frame-major, each frame row-major with x fastest. Pixel index p = y*nx + x.
 *  - Transposes of complex data are conjugate transposes (R is Hermitian).
 *  - Window grid: subset d = a*gx + b, centre ((a+1/2)*ny/gy - 1/2, (b+1/2)*nx/gx - 1/2),
 *    sigma = sigma_frac * spacing per axis, value exp(-dy^2/2sy^2 - dx^2/2sx^2),
 *    zero outside the box |y - cy| <= trunc_sigmas*sy, |x - cx| <= trunc_sigmas*sx.
 *    sigma_frac == 0 with a 1x1 grid is the flat window (global processing).
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees them. All launches go to `stream` (a hipStream_t; NULL = the
 *    default stream) and are asynchronous: a call returns once work is queued.
 *  - Argument errors are reported synchronously, before any launch, and leave
 *    the outputs untouched. Device-side conditions (non-finite input, Jacobi
 *    sweep cap, degenerate spectrum) set per-subset flags that lcf_sync reports.
 *  - A context is bound to one device; it is not thread-safe. It owns the
 *    scratch arena (grown on demand, reused afterwards), plans and MLP weights.
 *  - Stream capture: lcf_filter, lcf_filter_noalloc, lcf_filter_batch,
 *    lcf_stream_push, lcf_heevd_batched, lcf_mlp_infer and lcf_mlp_train_step
 *    return LCF_ERR_UNSUPPORTED, before any
 *    launch, when `stream` is being captured into a graph by the caller (they
 *    upload plans and may grow the arena, which a later call would overwrite or
 *    free under the caller's graph). With LCF_OPT_USE_GRAPH the library captures
 *    and replays its own graphs instead.
 */
#ifndef LCF_H
#define LCF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LCF_ABI_VERSION 6

typedef enum {
    LCF_OK = 0,
    LCF_ERR_INVALID_ARG = 1,     /* bad sizes, NULL pointers, unknown enum values      */
    LCF_ERR_UNSUPPORTED = 2,     /* valid but not implemented (e.g. nt > 208)           */
    LCF_ERR_OUT_OF_MEMORY = 3,   /* arena growth failed                                 */
    LCF_ERR_DEVICE = 4,          /* a HIP call failed                                   */
    LCF_ERR_NONFINITE_INPUT = 5, /* reported by lcf_sync: NaN/Inf reached a covariance  */
    LCF_ERR_NO_CONVERGENCE = 6,  /* reported by lcf_sync: Jacobi hit the sweep cap      */
    LCF_ERR_MODEL = 7,           /* MLP weights missing or checkpoint corrupt           */
    LCF_ERR_SCRATCH_LIMIT = 8    /* lcf_filter_noalloc: the call's workspace exceeds
                                    LCF_NOALLOC_SCRATCH_BYTES                           */
} lcf_status;

/* Arithmetic of the covariance and reprojection GEMMs. Both keep FP64 for the
 * eigen-solve and for the rank-r tissue part that needs it. */
typedef enum {
    LCF_PREC_FP32 = 0,   /* FP32 MFMA, FP32 accumulate                              */
    LCF_PREC_BF16X3 = 1  /* split BF16 (x = hi + lo, three products), FP32 accumulate */
} lcf_precision;

typedef enum {
    LCF_CUT_FIXED_K = 0,  /* k = k_fixed (Eq. 4)                                     */
    LCF_CUT_KNEE = 1,     /* k = argmax curvature of the log-eigenvalue curve (Eq. 6) */
    LCF_CUT_EXPLICIT = 2, /* caller's weights explicit_w[d][i]                       */
    LCF_CUT_MLP = 3,      /* weights from the context's MLP (needs Nt = 128)          */
    LCF_CUT_MEDIAN = 4,   /* k = #{i : lambda_i > beta_median * lambda_median} (Eq. 7) */
    LCF_CUT_SLOPE = 5,    /* k = first n with |slope| <= slope_thr (method 2, Fig. 2c) */
    LCF_CUT_POWER = 6,    /* soft w_i = win(i) / lambda_i^beta_power, max 1 (Eq. 10)   */
    LCF_CUT_NCC = 7       /* method 4 (Eq. 8): k = smallest 1-based index of the minimum
                             over k in [5, Nt - 5] of NCC(I_T(k), I_B(k)), with
                             I_T(k) = sum_{i=k-4..k} |u_i|, I_B(k) = sum_{i=k+1..k+5} |u_i|
                             per pixel of the windowed subset, u_i = C_w v_i / sqrt(lambda_i)
                             (0 where lambda_i <= 0), NCC(a, b) = sum ab / (|a| |b|) with
                             no mean removed; no value anywhere (all images zero, or
                             Nt < 10) gives k = 0 and LCF_FLAG_NONPOSITIVE. With
                             LCF_SHAPE_SIGMOID this is method 5 (Eq. 9 on that k).
                             Needs every eigenvector and the scores of every pixel: an
                             FP64 product of the size of the projection, about as slow
                             as the rest of the filter                              */
} lcf_cut;

typedef enum {
    LCF_SHAPE_HARD = 0,    /* w_i = 0 for i <= k, else 1 (Eq. 4)                     */
    LCF_SHAPE_SIGMOID = 1  /* w_i = 1 / (1 + exp(-beta_sigmoid (i - k))) (Eq. 9)     */
} lcf_shape;

typedef enum {
    LCF_PD_EQ13 = 0,             /* alpha_d = Npix*Nt / sum_i w_i^2 lambda_i (Eq. 13)   */
    LCF_PD_SUM = 1,              /* alpha_d = 1                                         */
    LCF_PD_EQ13_COMPENSATED = 2  /* Eq. 13, then divided by sum_d alpha_d w_d(x)^2      */
} lcf_pd_mode;

/* Packet shape and window grid (Eq. 11, Fig. 3). */
typedef struct {
    int32_t ny, nx, nt;      /* packet dims; 4 <= nt <= 208, ny*nx <= 2^26               */
    int32_t gy, gx;          /* window grid; gy <= ny, gx <= nx                          */
    int32_t reserved;        /* must be 0                                               */
    double sigma_frac;       /* sigma = sigma_frac * spacing per axis (1/3 typical);
                                0 = flat window, requires gy = gx = 1                   */
    double trunc_sigmas;     /* box half-width in sigmas (6 typical); 0 = whole image   */
} lcf_geometry;

/* Thresholding rule (Adaptive Thresholding Methods section). */
typedef struct {
    int32_t cut;             /* lcf_cut                                                  */
    int32_t shape;           /* lcf_shape (ignored for EXPLICIT, MLP and POWER)          */
    int32_t pd_mode;         /* lcf_pd_mode                                              */
    int32_t k_fixed;         /* FIXED_K: 0 <= k_fixed <= nt                               */
    double beta_knee;        /* Eq. 6 normalisation factor beta (> 0), typically 1        */
    double knee_max_frac;    /* curvature search over n in [2, floor(frac*nt)], (0, 1]    */
    double beta_sigmoid;     /* Eq. 9 sharpness (> 0), e.g. 2                             */
    double deflate_rho;      /* tissue-deflation threshold (relative eigenvalue); 1e-5
                                typical; 0 disables the deflation (precision drops)     */
    const float* explicit_w; /* EXPLICIT: device float [nsubsets][nt], else NULL          */
    double beta_median;      /* MEDIAN: Eq. 7 scaling factor beta (> 0, finite); the median
                                of an even number of eigenvalues is the mean of the two
                                middle ones, and lambda_i equal to the threshold is kept */
    double slope_thr;        /* SLOPE: threshold (> 0, finite) on |y'(n)| of the curve
                                y(n) = Nt lambda_n / lambda_1, differences as for Eq. 6;
                                k = 0-based index of the first n with |y'(n)| <= slope_thr
                                (Nt if none); lambda_1 <= 0 sets NONPOSITIVE and k = 0 */
    double beta_power;       /* POWER: Eq. 10 order beta (> 0, finite); win(i) =
                                exp(-(2.5 i / (Nt - 1))^2 / 2), eigenvalues floored at
                                lambda_1 2^-52, weights scaled to a maximum of 1;
                                lambda_1 <= 0 sets NONPOSITIVE with all-ones weights  */
} lcf_threshold;

/* Optional per-subset diagnostics (device pointers, each may be NULL).
 * nd = gy*gx subsets per packet. */
typedef struct {
    double* eigvals;   /* [nd][nt]  eigenvalues of R_d, descending                        */
    float* weights;    /* [nd][nt]  eigencomponent weights w_i                           */
    int32_t* k;        /* [nd]      cut index (FIXED_K/KNEE/MEDIAN/SLOPE), -1 otherwise   */
    int32_t* sweeps;   /* [nd]      Jacobi sweeps used                                    */
    int32_t* flags;    /* [nd]      LCF_FLAG_* bits                                       */
    double* alpha;     /* [nd]      Eq. 13 subset weight                                  */
    double* cov;       /* [nd][nt][nt] complex128 (interleaved), R_d row-major            */
    double* eigvecs;   /* [nd][nt][nt] complex128, eigenvector j in column j              */
    int32_t* rank;     /* [nd]      number of tissue components deflated                  */
    double* curve;     /* [nd][nt]  LCF_CUT_NCC: the Eq. 8 curve, entry k-1 for 1-based k,
                                    NaN where it has no value; untouched for other cuts    */
    double* mlp_gate;  /* [nd]      LCF_CUT_MLP: the gate's predicted power Doppler deviation
                                    (dB) of the network's weights from the rule's (see
                                    LCF_OPT_MLP_GATE); +inf where the network was not
                                    applicable; untouched for other cuts                   */
} lcf_diag;

#define LCF_FLAG_NONPOSITIVE   1  /* lambda_1 <= 0 or log10(lambda_1) == 0 under KNEE: k = 0 */
#define LCF_FLAG_NONFINITE     2  /* NaN/Inf in the covariance                              */
#define LCF_FLAG_NO_CONVERGE   4  /* Jacobi reached max sweeps                               */
#define LCF_FLAG_MLP_FALLBACK  8  /* learned weights not used, rule weights kept: input out of
                                     range, or the gate (LCF_OPT_MLP_GATE) rejected them    */
#define LCF_FLAG_EVD_JACOBI   16  /* near-degenerate pair at a component the projector needs
                                     (weight != 1, or every component under the NCC rule or
                                     when the diagnostics ask for all eigenvectors): EVD by
                                     Jacobi instead of the tridiagonal solver (informational) */

/* Context options (lcf_set_option). */
#define LCF_OPT_SCHEDULE     1  /* 0 = batched (all subsets per stage in one launch, default);
                                   1 = sequential: the paper's per-subset loop (Discussion),
                                   one launch chain per subset                              */
#define LCF_OPT_MAX_SWEEPS   2  /* Jacobi sweep cap (default 30)                            */
#define LCF_OPT_USE_GRAPH    3  /* 1 = capture the launch chain in a hipGraph and replay it
                                   for repeated calls with the same plan (default 0)       */
#define LCF_OPT_SUBSPACE_IT  4  /* subspace iterations for the tissue basis (default 3)     */
#define LCF_OPT_STAGE_TIMING 5  /* 1 = bracket every kernel launch with HIP events on the
                                   caller's stream and accumulate per-stage device time
                                   (read with lcf_stage_time; default 0)                  */
#define LCF_OPT_AUTOTUNE     6  /* 1 = before the first call of a launch-group class (padded
                                   Nt, precision, schedule, log2 subset count, log2 mean
                                   box size) with no stored choice, time every split-K
                                   chunk {512..4096 px} x reprojection kernel (tiles of
                                   2 or 4 rows; with 4 rows, all waves alike or split
                                   into producer and consumer waves)
                                   on the call's own packets and keep the fastest, then,
                                   up to 128 frames, the other subset EVD method
                                   (LCF_OPT_EVD values) on the winning plan
                                   (default 0: 1024 px, 4 rows up to 128 frames, else 2;
                                   producer/consumer waves for FP32 only; the context's
                                   EVD method). Tuning is skipped while the stream is
                                   being captured.                                        */

#define LCF_OPT_EVD          7  /* subset EVD (Eq. 2) up to 128 frames: 0 = Householder
                                   tridiagonal reduction, multisection eigenvalues and
                                   twisted-factorisation eigenvectors, with the Jacobi
                                   solver for subsets where a component whose vector the
                                   projector needs has a neighbour closer than 1e-12
                                   lambda_1 (flag LCF_FLAG_EVD_JACOBI; default);
                                   1 = FP64 one-sided Jacobi for every subset           */

#define LCF_OPT_MLP_GATE     8  /* learned weights: the plain rule (the threshold's curvature
                                   rule and shape) is the fallback and the judge. A subset
                                   keeps the rule's weights (LCF_FLAG_MLP_FALLBACK) when the
                                   predicted power Doppler deviation of the network's weights
                                   from the rule's is at least this many milli-dB (default
                                   100 = 0.1 dB; 0 = always the rule; -1 = no gate). The
                                   prediction: after Eq. 13 each subset's power Doppler at a
                                   pixel is a mixture, over components, of the same pixel
                                   profiles weighted by each component's share of the
                                   filtered energy, so the ratio of the two images lies
                                   between the extreme share ratios of the components
                                   present; the largest |10 log10| share ratio over the
                                   components holding at least 0.1% of either energy    */

/* Kernel stages reported by lcf_stage_time. */
typedef enum {
    LCF_STAGE_WINDOWS = 0,      /* Gaussian window factors (Eq. 11)                       */
    LCF_STAGE_GRAM1 = 1,        /* windowed covariance, split-K MFMA (Eq. 12)             */
    LCF_STAGE_GRAM1_REDUCE = 2, /* ordered FP64 reduction of the split-K partials          */
    LCF_STAGE_TISSUE = 3,       /* tissue basis for the deflation                          */
    LCF_STAGE_GRAM2 = 4,        /* covariance of the deflated data [C' | C_w V_r]          */
    LCF_STAGE_GRAM2_REDUCE = 5,
    LCF_STAGE_ASSEMBLE = 6,     /* R from the deflated Gram, B = Q^H R Q                   */
    LCF_STAGE_EVD = 7,          /* FP64 subset EVD (Eq. 2): tridiagonal solver or Jacobi   */
    LCF_STAGE_RULES = 8,        /* eigencomponent weights (Eqs 4, 6, 9), alpha (Eq. 13)    */
    LCF_STAGE_MLP = 9,          /* learned weights                                         */
    LCF_STAGE_PROJECTOR = 10,   /* P = V diag(w) V^H                                       */
    LCF_STAGE_REPROJ = 11,      /* projection, power Doppler, recombination (Eqs 4, 13)    */
    LCF_STAGE_EVD_VECTORS = 12, /* eigenvectors of the weighted components (tridiagonal solver) */
    LCF_STAGE_NCC = 13,         /* method 4 scores and curve sums (Eq. 8)                  */
    LCF_STAGE_COV_STREAM = 14,  /* sliding packets: FP64 covariance update by the hop      */
    LCF_NUM_STAGES = 15
} lcf_stage;

typedef struct lcf_context lcf_context;

/* Create a context on HIP device `device`. *out receives the handle. */
lcf_status lcf_create(int32_t device, lcf_context** out);
/* Release the context and its device memory. NULL is accepted. Everything is
 * released even when a HIP call fails on the way (after an earlier device
 * fault, say); the return is then LCF_ERR_DEVICE. */
lcf_status lcf_destroy(lcf_context* ctx);
/* Set a context option (LCF_OPT_*). */
lcf_status lcf_set_option(lcf_context* ctx, int32_t option, int64_t value);

/* Host-only validation of a geometry/threshold/precision triple (no GPU needed).
 * Returns LCF_OK or the error lcf_filter would return for these arguments. */
lcf_status lcf_validate(const lcf_geometry* geo, const lcf_threshold* thr, int32_t precision);

/* Filter one packet (Eqs 1-13, Localized Clutter Filtering section).
 *   iq      device complex64 [nt][ny][nx]                     (input, not modified)
 *   iq_out  device complex64 [nt][ny][nx] or NULL: sum_d Chat_d / sum_d w_d
 *   pd      device float [ny][nx]: power Doppler after Eq. 13 recombination
 *   diag    optional diagnostics (host struct holding device pointers), or NULL */
lcf_status lcf_filter(lcf_context* ctx, const lcf_geometry* geo, const lcf_threshold* thr,
                      int32_t precision, const void* iq, void* iq_out, float* pd,
                      const lcf_diag* diag, void* stream);

/* Allocation-free variant of lcf_filter, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels, results and errors as lcf_filter, except that the
 * plan descriptors, the workspace and the network activations of the call live
 * in one fixed device block of LCF_NOALLOC_SCRATCH_BYTES that the library
 * holds per device for the life of the process (set up by lcf_create), and
 * that the call allocates no device or pinned host memory: it never grows the
 * context's arena, never autotunes (a choice already stored in the context is
 * used) and never captures a graph. A call whose workspace does not fit
 * returns LCF_ERR_SCRATCH_LIMIT before any launch (a 256 x 192 x 128 packet
 * with an 8 x 8 grid fits; a 512 x 256 x 128 packet with a 16 x 16 grid does
 * not). Plan uploads are staged in the context's host memory (C++ heap, grown
 * once to the largest plan). All calls on one device share the block and
 * every call overwrites it: calls that may overlap on one device (other
 * streams, other contexts, other threads) race and must be serialised by the
 * caller; calls on one stream are ordered. Refused under stream capture like
 * lcf_filter. */
#define LCF_NOALLOC_SCRATCH_BYTES (192u * 1024u * 1024u)
lcf_status lcf_filter_noalloc(lcf_context* ctx, const lcf_geometry* geo, const lcf_threshold* thr,
                              int32_t precision, const void* iq, void* iq_out, float* pd,
                              const lcf_diag* diag, void* stream);

/* Filter n packets of possibly different shapes and grids in one batched pass
 * (the parallel processing of subsets that the Discussion leaves for future work).
 * geo[n] host array; iq/iq_out/pd are host arrays of n device pointers (iq_out[i]
 * may be NULL, iq_out itself may be NULL). One threshold rule applies to all.
 * n >= 1: an empty batch returns LCF_ERR_INVALID_ARG. Caller-given weights
 * (LCF_CUT_EXPLICIT): thr->explicit_w holds each packet's [nd_i][nt_i] block,
 * packets back to back in call order (sum_i nd_i nt_i floats). */
lcf_status lcf_filter_batch(lcf_context* ctx, int32_t n, const lcf_geometry* geo,
                            const lcf_threshold* thr, int32_t precision,
                            const void* const* iq, void* const* iq_out, float* const* pd,
                            void* stream);

/* ---- sliding packets --------------------------------------------------------
 * The paper processes packets that slide over a recording by a few frames
 * (Experimental Studies section: a 5-frame hop; Discussion: display rate).
 * Consecutive packets share every frame pair but the new ones, so the covariance
 * of each window (Eq. 12) is carried from one packet to the next: the entries
 * between retained frames are moved by the hop and only the hop new columns
 * are summed over the window's box, in FP64 from the FP32 packet values (no
 * subtraction, so nothing drifts). The FP64 covariance replaces both Gram
 * passes of lcf_filter (it gives the tissue basis and B = Q^H R Q directly);
 * the weights, projection, power Doppler and recombination are lcf_filter's.
 *
 * lcf_stream_create: one stream of packets of one geometry, rule and precision
 *   (arguments as lcf_filter; the threshold is copied, its explicit_w pointer
 *   kept). The stream owns two FP64 covariance buffers (nd * nt^2 complex128
 *   each, nt padded) and the partial sums of the new columns; everything else
 *   comes from the context's arena. *out receives the handle.
 * lcf_stream_push: filter the current packet iq (device complex64
 *   [nt][ny][nx]; e.g. a pointer into a longer recording [T][ny][nx] advanced
 *   by hop frames per push) whose first nt - hop frames are the last nt - hop
 *   frames of the previous push's packet (the caller's contract: it is not
 *   checked). 1 <= hop <= nt; the first push after create computes every
 *   column whatever hop says. iq_out, pd and diag as lcf_filter; calls on one
 *   stream must be made in packet order on one HIP stream.
 * lcf_stream_destroy: release the stream's buffers (waits for the device);
 *   as lcf_destroy, everything is released and a failed HIP call on the way
 *   returns LCF_ERR_DEVICE. */
typedef struct lcf_stream lcf_stream;
lcf_status lcf_stream_create(lcf_context* ctx, const lcf_geometry* geo, const lcf_threshold* thr,
                             int32_t precision, lcf_stream** out);
lcf_status lcf_stream_push(lcf_stream* s, const void* iq, int32_t hop, void* iq_out, float* pd,
                           const lcf_diag* diag, void* stream);
lcf_status lcf_stream_destroy(lcf_stream* s);

/* Batched Hermitian eigen-decomposition (Eq. 2) with the library's FP64 one-sided
 * Jacobi: a = device complex128 [n][nt][nt] (row-major, Hermitian; only read),
 * w = device double [n][nt] eigenvalues descending, v = device complex128
 * [n][nt][nt] with eigenvector j in column j (may be NULL), sweeps = device
 * int32 [n] (may be NULL). 2 <= nt <= 256. */
lcf_status lcf_heevd_batched(lcf_context* ctx, int32_t n, int32_t nt, const double* a,
                             double* w, double* v, int32_t* sweeps, void* stream);

/* ---- learned eigencomponent weights ----------------------------------------
 * A 128-256-256-128 MLP (GELU, GELU, sigmoid) maps a subset's normalised
 * log-eigenvalue spectrum z_i = log10(max(lambda_i, lambda_1 2^-52)/lambda_1)/8
 * to soft weights w_i for the projection of Eq. 4 (the role the threshold
 * rules of Eqs 6 and 9 play). Parameters (FP32 master, BF16 working copy, Adam
 * moments) live in the context. Parameter order: W1[256][128], b1[256],
 * W2[256][256], b2[256], W3[128][256], b3[128] (row-major, out x in).
 * With LCF_CUT_MLP, lcf_filter first applies the curvature rule with the
 * threshold's shape and betas (the fallback), then replaces the weights of
 * every subset whose Nt is 128 and whose spectrum is finite and positive;
 * the others keep the rule and get LCF_FLAG_MLP_FALLBACK. */
#define LCF_MLP_NPARAM 131712

/* Initialise the parameters from `seed` (uniform, scaled by fan-in). */
lcf_status lcf_mlp_init(lcf_context* ctx, uint64_t seed);
/* Copy n = LCF_MLP_NPARAM FP32 parameters in from / out to host memory. */
lcf_status lcf_mlp_set_params(lcf_context* ctx, const float* host, int64_t n);
lcf_status lcf_mlp_get_params(lcf_context* ctx, float* host, int64_t n);
/* Gradients of the last lcf_mlp_train_step (same order), to host memory. */
lcf_status lcf_mlp_get_grads(lcf_context* ctx, float* host, int64_t n);
/* Checkpoint: magic, version, sizes, step, FP32 master + Adam moments, CRC32.
 * lcf_mlp_load returns LCF_ERR_MODEL on a bad magic, size or CRC and leaves the
 * current parameters untouched. */
lcf_status lcf_mlp_save(lcf_context* ctx, const char* path);
lcf_status lcf_mlp_load(lcf_context* ctx, const char* path);
/* Inference on b spectra: lam device double [b][128] (descending), w device
 * float [b][128]. */
lcf_status lcf_mlp_infer(lcf_context* ctx, const double* lam, float* w, int32_t b, void* stream);
/* One Adam step (lr, betas 0.9/0.999, eps 1e-8) on b spectra with targets
 * target (device float [b][128]); loss_out (device float, may be NULL) gets the
 * batch-mean loss sum_i c_i (w_i - t_i)^2, c_i = lambda_i / sum_j lambda_j t_j^2. */
lcf_status lcf_mlp_train_step(lcf_context* ctx, const double* lam, const float* target, int32_t b, float lr,
                              float* loss_out, void* stream);

/* Wait for `stream` and report the first device-side condition raised since
 * the previous lcf_sync (LCF_ERR_NONFINITE_INPUT, LCF_ERR_NO_CONVERGENCE). */
lcf_status lcf_sync(lcf_context* ctx, void* stream);

/* Accumulated device time (ms) and launch count of one stage since the last
 * reset, over the calls made with LCF_OPT_STAGE_TIMING = 1. Waits for the
 * recorded events. reset != 0 clears all stages after reading. */
lcf_status lcf_stage_time(lcf_context* ctx, int32_t stage, double* ms, int64_t* launches, int32_t reset);

/* Autotuner choices (batched form of many packets and subsets, Discussion:
 * parallel processing of subsets) as text, one line per launch-group class:
 * "<class> <chunk> <rows> <variant> <evd>" (evd: 0 tridiagonal, 1 Jacobi, -1 the
 * context's LCF_OPT_EVD; lines without it are read as -1). lcf_tune_save writes the context's choices to `path`;
 * lcf_tune_load adds the choices in `path` to the context (replacing entries of
 * the same class) and drops captured graphs. Errors: LCF_ERR_INVALID_ARG for
 * NULL arguments, an unreadable/unwritable file or a malformed line (nothing is
 * loaded from a file with a malformed line). */
lcf_status lcf_tune_save(lcf_context* ctx, const char* path);
lcf_status lcf_tune_load(lcf_context* ctx, const char* path);

const char* lcf_status_str(lcf_status s);
int32_t lcf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LCF_H */
