// Eigencomponent weights (Eqs 4, 6, 7, 9, 10, slope rule), the projector P = V diag(w) V^H, and
// the output-centric reprojection + power Doppler + recombination (Eqs 4, 5, 13).
#include "lcf_internal.h"
#include "lcf_kernels.h"

namespace lcf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even FP32 -> BF16 bits.
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// ------------------------------------------------------------------ rules
// One 64-lane wave per subset; everything on the FP64 eigenvalues.
__global__ void __launch_bounds__(64) k_rules(Workspace ws, RuleParams rp) {
    __shared__ double yt[256], d1[256], kv[256];
    __shared__ int sh_k, sh_flag;
    const int s = blockIdx.x, lane = threadIdx.x;
    const SubsetDesc sd = ws.sub[s];
    const int nt = sd.nt, ntp = ws.ntp;
    const double* lam = ws.lam + (long)s * ntp;
    double* wts = ws.wts + (long)s * ntp;
    if (lane == 0) { sh_k = -1; sh_flag = 0; }
    __syncthreads();
    if (rp.cut == 0 || rp.cut == 1 || rp.cut == 4 || rp.cut == 5 || rp.cut == 7) {
        int k = rp.k_fixed;
        if (rp.cut == 7) {
            // method 4 (Eq. 8): add the chunk partials of the three curve sums in
            // chunk order, NCC(k) = sum I_T I_B / (sqrt(sum I_T^2) sqrt(sum I_B^2)) over
            // 1-based k in [fn, nt - fn] (NaN elsewhere and where an image is zero);
            // k = smallest index of the minimum, 0 and NONPOSITIVE when none has a value
            constexpr int FN = 5;
            const double* part = (const double*)ws.partial;
            const int c0 = ws.chunk_begin[s], c1 = ws.chunk_begin[s + 1];
            double* curve = ws.curve + (long)s * ntp;
            double best = INFINITY;
            int bi = 1 << 30;
            for (int i = lane; i < ntp; i += 64) {
                const int k1 = i + 1;
                double v = NAN;
                if (k1 >= FN && k1 <= nt - FN) {
                    double tb = 0.0, tt = 0.0, bb = 0.0;
                    for (int c = c0; c < c1; ++c) {
                        tb += part[(long)c * 3 * ntp + i];
                        tt += part[(long)c * 3 * ntp + ntp + i];
                        bb += part[(long)c * 3 * ntp + 2 * ntp + i];
                    }
                    const double den = sqrt(tt) * sqrt(bb);
                    if (den > 0.0) v = tb / den;
                }
                curve[i] = v;
                if (v < best) { best = v; bi = k1; }
            }
            for (int m = 32; m >= 1; m >>= 1) {
                const double ob = __shfl_xor(best, m, 64);
                const int oi = __shfl_xor(bi, m, 64);
                if (ob < best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (bi == (1 << 30)) {
                k = 0;
                if (lane == 0) sh_flag = 1;
            } else {
                k = bi;
            }
        }
        if (rp.cut == 5) {
            // slope rule: y(n) = Nt lambda_n / lambda_1, slopes by the differences
            // of the curvature rule; k = first 0-based n with |y'(n)| <= threshold
            const double l1 = lam[0];
            if (!(l1 > 0.0)) {
                k = 0;
                if (lane == 0) sh_flag = 1;
            } else {
                for (int i = lane; i < nt; i += 64) yt[i] = (double)nt * lam[i] / l1;
                __syncthreads();
                int first = nt;
                for (int i = lane; i < nt; i += 64) {
                    const double d = i == 0 ? yt[1] - yt[0]
                                            : (i == nt - 1 ? yt[nt - 1] - yt[nt - 2] : 0.5 * (yt[i + 1] - yt[i - 1]));
                    if (fabs(d) <= rp.slope_thr && i < first) first = i;
                }
                for (int m = 32; m >= 1; m >>= 1) first = min(first, __shfl_xor(first, m, 64));
                k = first;
            }
        }
        if (rp.cut == 4) {
            // Eq. 7: threshold beta times the median eigenvalue (lam is sorted
            // descending; an even count takes the mean of the two middle values);
            // k counts the eigenvalues strictly above it
            const int h = nt >> 1;
            const double med = (nt & 1) ? lam[h] : 0.5 * (lam[h - 1] + lam[h]);
            const double tval = rp.beta_median * med;
            int cnt = 0;
            for (int i = lane; i < nt; i += 64) cnt += lam[i] > tval ? 1 : 0;
            for (int m = 32; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m, 64);
            k = cnt;
        }
        if (rp.cut == 1) {
            const double l1 = lam[0];
            bool bad = !(l1 > 0.0);
            double y1 = 0.0;
            if (!bad) { y1 = log10(l1); bad = (y1 == 0.0); }
            if (bad) {
                k = 0;
                if (lane == 0) sh_flag = 1;
            } else {
                const double floor_ = l1 * 2.220446049250313e-16;     // lambda_1 * 2^-52
                for (int i = lane; i < nt; i += 64) {
                    const double l = lam[i] > floor_ ? lam[i] : floor_;
                    yt[i] = rp.beta_knee * (double)nt * log10(l) / y1;
                }
                __syncthreads();
                for (int i = lane; i < nt; i += 64)
                    d1[i] = i == 0 ? yt[1] - yt[0] : (i == nt - 1 ? yt[nt - 1] - yt[nt - 2] : 0.5 * (yt[i + 1] - yt[i - 1]));
                __syncthreads();
                for (int i = lane; i < nt; i += 64) {
                    const double d2 = i == 0 ? d1[1] - d1[0] : (i == nt - 1 ? d1[nt - 1] - d1[nt - 2] : 0.5 * (d1[i + 1] - d1[i - 1]));
                    kv[i] = fabs(d2) / pow(1.0 + d1[i] * d1[i], 1.5);
                }
                __syncthreads();
                int hi = (int)floor(rp.knee_max_frac * (double)nt);
                if (hi < 2) hi = 2;
                if (hi > nt) hi = nt;
                // smallest argmax over 0-based i in [1, hi-1]
                double best = -1.0;
                int bi = 1 << 30;
                for (int i = 1 + lane; i < hi; i += 64) {
                    if (kv[i] > best) { best = kv[i]; bi = i; }
                }
                for (int m = 32; m >= 1; m >>= 1) {
                    const double ob = __shfl_xor(best, m, 64);
                    const int oi = __shfl_xor(bi, m, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                k = bi + 1;
            }
        }
        if (lane == 0) sh_k = k;
        for (int i = lane; i < nt; i += 64) {
            const double n1 = (double)(i + 1);
            wts[i] = rp.shape == 0 ? (n1 > (double)k ? 1.0 : 0.0)
                                   : 1.0 / (1.0 + exp(-rp.beta_sigmoid * (n1 - (double)k)));
        }
    } else if (rp.cut == 6) {
        // Eq. 10: w_i = win(i) / lambda_i^beta with the half Gaussian window
        // win(i) = exp(-(2.5 i / (Nt - 1))^2 / 2), scaled to a maximum of 1; taken
        // in logarithms so that no power overflows
        const double l1 = lam[0];
        if (!(l1 > 0.0)) {
            for (int i = lane; i < nt; i += 64) wts[i] = 1.0;
            if (lane == 0) sh_flag = 1;
        } else {
            const double floor_ = l1 * 2.220446049250313e-16;     // lambda_1 * 2^-52
            double mx = -INFINITY;
            for (int i = lane; i < nt; i += 64) {
                const double l = lam[i] > floor_ ? lam[i] : floor_;
                const double u = 2.5 * (double)i / (double)(nt - 1);
                const double lw = -0.5 * u * u - rp.beta_power * log(l);
                yt[i] = lw;
                mx = fmax(mx, lw);
            }
            for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m, 64));
            for (int i = lane; i < nt; i += 64) wts[i] = exp(yt[i] - mx);
        }
    } else if (rp.cut == 2) {
        for (int i = lane; i < nt; i += 64) wts[i] = (double)ws.explicit_w[sd.ew_off + i];
    } else {
        // weights already written by the MLP kernel
    }
    for (int i = nt + lane; i < ntp; i += 64) wts[i] = 0.0;
    __syncthreads();
    double e = 0.0;
    for (int i = lane; i < nt; i += 64) e += wts[i] * wts[i] * lam[i];
    e = wave_sum(e);
    if (lane == 0) {
        ws.kcut[s] = (rp.cut <= 1 || rp.cut == 4 || rp.cut == 5 || rp.cut == 7) ? sh_k : -1;
        ws.alpha[s] = rp.pd_mode == 1 ? 1.0 : (e > 0.0 ? sd.npix_nt / e : 0.0);
        if (sh_flag) atomicOr(&ws.flags[s], sh_flag);
    }
}

// Within every block of 16 frames the split-BF16 operand rows are stored in the
// order of the FP64 residual's accumulator layout: position 4 g + e holds frame
// g + 4 e (a 4 x 4 transpose, its own inverse), so each lane of the residual
// stores four consecutive positions at once.
__host__ __device__ constexpr int sb_perm16(int x) { return (x & ~15) | ((x & 3) << 2) | ((x >> 2) & 3); }

// Split-BF16 [P; M] operand planes (layout described at k_reproj_sb): the KC
// rows of P, padded to whole K steps of 32, then a 32-row packed block for M.
template <int NTP>
struct SbLayout {
    static constexpr int KC = (NTP + 31) / 32 * 32;    // rows of P per plane row, whole K steps
    static constexpr int KB = KC + 32;                 // plane row length
};

// ------------------------------------------------------------------ projector
// With the eigenvectors W of B = Q^H R Q (Q = H_0 .. H_{r-1}) and the weights w,
// the projector of Eq. 4 in the original basis is
//   P = Q (I - W diag(1 - w) W^H) Q^H = I - W' diag(1 - w) W'^H,  W' = Q W,
// (exactly U diag(w) U^H on the range of B; all-ones weights give P = I). Only
// the columns with w != 1 enter. Since V_r = Q [e_0 .. e_{r-1}],
//   M = V_r^H P = V_r^H - W[0..r-1, :] diag(1 - w) W'^H.
// Per chunk of PCC columns: W' by the r reflectors (16 lanes per column), then
// the P block in registers (thread: 8 consecutive rows t x 8 columns u with
// stride 16, 128 x 128 per pass) and M in LDS; finally the real-form or
// split-BF16 [P; M] planes used by the reprojection GEMM.
constexpr int PCC = 16;

// From 96 frames up the 128 x 128 P blocks are spread over 512 threads (4 rows
// x 8 columns each): with 256 threads the 8 x 8 FP64 accumulators left room
// for one wave per SIMD only.
template <int NTP>
struct PjCfg {
    static constexpr int NTHR = NTP >= 96 ? 512 : 256;
    static constexpr int RA = 2048 / NTHR;      // rows per thread in a 128 x 128 block
};

template <int NTP, int PREC>
__global__ void __launch_bounds__(PjCfg<NTP>::NTHR) k_projector(Workspace ws) {
    constexpr int NTHR = PjCfg<NTP>::NTHR, RA = PjCfg<NTP>::RA, NWV = NTHR / 64;
    constexpr int NTE = NTP + REXT;
    constexpr int KC = SbLayout<NTP>::KC, KB = SbLayout<NTP>::KB;
    constexpr int NB = (NTP + 127) / 128;       // 128 x 128 blocks per dimension
    constexpr int RW = NTP / 16;                // rows per lane in the reflector pass
    __shared__ double2 Wl[PCC * NTP];           // chunk of W, then W', [c][t]
    __shared__ double2 vh[RMAX * NTP];          // reflectors [j][t]
    __shared__ double2 Msh[RMAX * NTP];         // M [j][n]
    __shared__ double2 Wj[RMAX * PCC];          // rows 0 .. r-1 of the chunk of W
    __shared__ double cw[PCC];
    __shared__ double tau[RMAX];
    __shared__ int act[NTP];
    __shared__ int wcnt[NWV];
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = ws.sub[s].nt;
    const int r = ws.rank[s];
    const double2* W = ws.bmat + (long)s * NTP * NTP;        // column-major eigenvectors
    const double* wts = ws.wts + (long)s * NTP;

    // active columns (w != 1) in ascending order, by ballots
    const bool flag = tid < nt && fabs(1.0 - wts[tid < NTP ? tid : 0]) > 1e-17;
    const unsigned long long mask = __ballot(flag);
    if (lane == 0) wcnt[wave] = __popcll(mask);
    for (int e = tid; e < RMAX * NTP; e += NTHR) {
        const int j = e / NTP, t = e % NTP;
        vh[e] = j < r ? ws.hv[((long)s * RMAX + j) * NTP + t] : make_double2(0.0, 0.0);
        // M starts from V_r^H (zero beyond nt and r)
        Msh[e] = (j < r && t < nt) ? cconj(ws.vr64[((long)s * NTP + t) * RMAX + j]) : make_double2(0.0, 0.0);
    }
    if (tid < RMAX) tau[tid] = tid < r ? ws.htau[(long)s * RMAX + tid] : 0.0;
    __syncthreads();
    int nact = 0, off = 0;
    for (int w = 0; w < NWV; ++w) {
        off += w < wave ? wcnt[w] : 0;
        nact += wcnt[w];
    }
    if (flag) act[off + __popcll(mask & ((1ull << lane) - 1ull))] = tid;
    __syncthreads();

    const int ti = tid >> 4, ui = tid & 15;
    for (int bb = 0; bb < NB * NB; ++bb) {
        const int tb = 128 * (bb / NB), ub = 128 * (bb % NB);
        double2 acc[RA][8];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = make_double2(0.0, 0.0);
        for (int c0 = 0; c0 < nact; c0 += PCC) {
            const int cn = nact - c0 < PCC ? nact - c0 : PCC;
            // W' of the chunk: column c by lanes 16 c .. 16 c + 15, rows l + 16 i
            // (threads 0 .. 255)
            if (tid < 16 * PCC) {
                const int c = tid >> 4, l = tid & 15;
                double2 x[RW];
#pragma unroll
                for (int i = 0; i < RW; ++i)
                    x[i] = c < cn ? W[(long)act[c0 + c] * NTP + l + 16 * i] : make_double2(0.0, 0.0);
                if (bb == 0 && l < RMAX) Wj[l * PCC + c] = x[0];
                for (int j = r - 1; j >= 0; --j) {
                    double dr = 0.0, di = 0.0;
#pragma unroll
                    for (int i = 0; i < RW; ++i) {
                        const double2 v = vh[j * NTP + l + 16 * i];
                        dr = fma(v.x, x[i].x, fma(v.y, x[i].y, dr));       // conj(v) x
                        di = fma(v.x, x[i].y, fma(-v.y, x[i].x, di));
                    }
                    // sum over the 16 lanes of the row (lane moves within it)
                    dr += dpp_d<0xB1>(dr);
                    di += dpp_d<0xB1>(di);
                    dr += dpp_d<0x4E>(dr);
                    di += dpp_d<0x4E>(di);
                    dr += dpp_d<0x141>(dr);
                    di += dpp_d<0x141>(di);
                    dr += dpp_d<0x140>(dr);
                    di += dpp_d<0x140>(di);
                    const double2 nd = make_double2(-tau[j] * dr, -tau[j] * di);
#pragma unroll
                    for (int i = 0; i < RW; ++i) x[i] = cfma(vh[j * NTP + l + 16 * i], nd, x[i]);
                }
#pragma unroll
                for (int i = 0; i < RW; ++i) Wl[c * NTP + l + 16 * i] = x[i];
                if (tid < PCC) cw[tid] = tid < cn ? 1.0 - wts[act[c0 + tid]] : 0.0;
            }
            __syncthreads();
            // P block: acc[a][b] -= cw_c W'[t_a][c] conj(W'[u_b][c])
            for (int c = 0; c < cn; ++c) {
                double2 wt[RA], wu[8];
#pragma unroll
                for (int a = 0; a < RA; ++a) {
                    const int t = tb + (PREC ? sb_perm16(RA * ti + a) : RA * ti + a);
                    wt[a] = t < NTP ? cscale(Wl[c * NTP + t], cw[c]) : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int u = ub + ui + 16 * b;
                    wu[b] = u < NTP ? Wl[c * NTP + u] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int a = 0; a < RA; ++a)
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        acc[a][b].x = fma(-wt[a].x, wu[b].x, fma(-wt[a].y, wu[b].y, acc[a][b].x));
                        acc[a][b].y = fma(-wt[a].y, wu[b].x, fma(wt[a].x, wu[b].y, acc[a][b].y));
                    }
            }
            // M once: M[j][n] -= sum_c W[j][c] (1 - w_c) conj(W'[n][c])
            if (bb == 0) {
                for (int e = tid; e < RMAX * NTP; e += NTHR) {
                    const int j = e / NTP, n = e % NTP;
                    if (j < r && n < nt) {
                        double2 m = Msh[e];
                        for (int c = 0; c < cn; ++c) {
                            const double2 q = cscale(Wj[j * PCC + c], cw[c]);
                            const double2 wn = Wl[c * NTP + n];
                            m.x -= fma(q.x, wn.x, q.y * wn.y);            // q conj(wn)
                            m.y -= fma(q.y, wn.x, -q.x * wn.y);
                        }
                        Msh[e] = m;
                    }
                }
            }
            __syncthreads();
        }
        // write the block: operand row k = t (split BF16: the thread's rows are
        // frames sb_perm16 of RA consecutive plane positions), output frame n = u;
        // P = I - ... on [0, nt) x [0, nt), zero elsewhere
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int n = ub + ui + 16 * b;
            if (n >= NTP) continue;
            float re[RA], im[RA];
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const int k = tb + (PREC ? sb_perm16(RA * ti + a) : RA * ti + a);   // frame
                const bool in = k < nt && n < nt;
                re[a] = in ? (float)((k == n ? 1.0 : 0.0) + acc[a][b].x) : 0.f;
                im[a] = in ? (float)acc[a][b].y : 0.f;
            }
            const int k0 = tb + RA * ti;
            if (k0 >= NTP) continue;
            if (PREC == 1) {
                uint16_t* pt = reinterpret_cast<uint16_t*>(ws.breal + (long)s * (2 * NTE) * (2 * NTP));
                uint32_t h[RA], l[RA];
#pragma unroll
                for (int a = 0; a < RA; ++a) split_bf16x2(re[a], im[a], h[a], l[a]);
                // RA consecutive positions of each plane: RA / 2 words
                uint32_t hr[RA / 2], lr[RA / 2], hi4[RA / 2], li4[RA / 2];
#pragma unroll
                for (int q = 0; q < RA / 2; ++q) {
                    hr[q] = __builtin_amdgcn_perm(h[2 * q + 1], h[2 * q], 0x05040100u);
                    lr[q] = __builtin_amdgcn_perm(l[2 * q + 1], l[2 * q], 0x05040100u);
                    hi4[q] = __builtin_amdgcn_perm(h[2 * q + 1], h[2 * q], 0x07060302u);
                    li4[q] = __builtin_amdgcn_perm(l[2 * q + 1], l[2 * q], 0x07060302u);
                }
                const long e = (long)n * KB + k0;
                auto put = [&](long plane, const uint32_t* w) {
                    if constexpr (RA == 8)
                        *reinterpret_cast<u32x4*>(pt + plane * NTP * KB + e) = u32x4{w[0], w[1], w[2], w[3]};
                    else
                        *reinterpret_cast<uint2*>(pt + plane * NTP * KB + e) = make_uint2(w[0], w[1]);
                };
                put(0, hr);
                put(1, lr);
                put(2, hi4);
                put(3, li4);
            } else {
                // real form: row k of [P; M] at k, its i-multiple at NTE + k
                float* Br = ws.breal + (long)s * (2 * NTE) * (2 * NTP);
#pragma unroll
                for (int a = 0; a < RA; ++a) {
                    const int k = k0 + a;
                    Br[(long)k * (2 * NTP) + n] = re[a];
                    Br[(long)k * (2 * NTP) + NTP + n] = im[a];
                    Br[(long)(NTE + k) * (2 * NTP) + n] = -im[a];
                    Br[(long)(NTE + k) * (2 * NTP) + NTP + n] = re[a];
                }
            }
        }
    }
    // rows [NTP, KC) of the planes are zero; rows [KC, KB) hold M packed as the
    // reprojection's 32-row block (Msh is zero from r and from nt up)
    if (PREC == 1) {
        static_assert(RMAX == 8 && KB - KC == 32, "four blocks of 8 tissue columns");
        uint16_t* pt = reinterpret_cast<uint16_t*>(ws.breal + (long)s * (2 * NTE) * (2 * NTP));
        for (int e = tid; e < NTP * (KB - NTP); e += NTHR) {
            const int n = e / (KB - NTP), k = NTP + e % (KB - NTP);
            uint32_t w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
            if (k >= KC) {
                const int blk = (k - KC) >> 3, j = (k - KC) & 7;
                const double2 v = Msh[j * NTP + n];
                uint32_t h, l;
                split_bf16x2((float)v.x, (float)v.y, h, l);
                const uint32_t hre = h & 0xffffu, him = h >> 16, lre = l & 0xffffu, lim = l >> 16;
                const bool odd = blk & 1, first = blk < 2;
                w0 = odd ? (him ^ 0x8000u) : hre;                      // [Mh_re | -Mh_im | Mh_re | -Mh_im]
                w1 = first ? (odd ? (lim ^ 0x8000u) : lre) : 0u;       // [Ml_re | -Ml_im | 0 | 0]
                w2 = odd ? hre : him;                                  // [Mh_im |  Mh_re | Mh_im |  Mh_re]
                w3 = first ? (odd ? lre : lim) : 0u;                   // [Ml_im |  Ml_re | 0 | 0]
            }
            const long o = (long)n * KB + k;
            pt[0L * NTP * KB + o] = (uint16_t)w0;
            pt[1L * NTP * KB + o] = (uint16_t)w1;
            pt[2L * NTP * KB + o] = (uint16_t)w2;
            pt[3L * NTP * KB + o] = (uint16_t)w3;
        }
    } else {
        float* Br = ws.breal + (long)s * (2 * NTE) * (2 * NTP);
        for (int e = tid; e < REXT * NTP; e += NTHR) {
            const int j = e / NTP, n = e % NTP;
            const double2 v = j < RMAX ? Msh[j * NTP + n] : make_double2(0.0, 0.0);
            const int k = NTP + j;
            Br[(long)k * (2 * NTP) + n] = (float)v.x;
            Br[(long)k * (2 * NTP) + NTP + n] = (float)v.y;
            Br[(long)(NTE + k) * (2 * NTP) + n] = -(float)v.y;
            Br[(long)(NTE + k) * (2 * NTP) + NTP + n] = (float)v.x;
        }
    }
}

// ------------------------------------------------------------------ reprojection
// One work-group per tile of TR image rows x TW pixels (output-centric
// gather, no atomics). For every covering subset d in ascending order:
//   y  = s V_r                      (FP64 partial sums, split over t, rounded to FP32)
//   c' = s - y V_r^H                (FP64, then rounded to the GEMM operand)
//   chat = [c' | y] [P; M]          (MFMA: FP32, or BF16 hi/lo with three products)
// and the epilogue accumulates in registers
//   PD(x)   += alpha_d w_d(x)^2 sum_t |chat(x, t)|^2     (Eq. 13)
//   IQ(x,t) += w_d(x) chat(x, t),  W(x) += w_d(x)
// The window factors out of the projection because C_hat_d(x, :) = w_d(x) s_x P_d.
// Each wave owns CTW output column tiles of all TP/16 pixel row tiles, so every
// [P; M] fragment read from memory serves TP pixels.
// Work-groups are mapped to tiles so that each of the 8 XCDs walks a contiguous
// range of tiles (neighbouring tiles share covering subsets, so their [P; M]
// operands are shared in that XCD's L2).
template <int NTP, int PREC, int TR>
struct RpCfg {
    static constexpr int TP = TR * TW;                                // pixels per tile
    static constexpr int NRT = TP / 16;                               // MFMA row tiles
    static constexpr int NTE = NTP + REXT;
    static constexpr int IMO = (NTE % 32 == 16) ? NTE : NTE + 16;     // FP32: offset of the im part
    static constexpr int LDA = 2 * IMO + 1;                           // FP32 row stride (floats)
    static constexpr int CT = (2 * NTP) / 16;                         // output column tiles
    static constexpr int NNT = NTP / 16;                              // output frame tiles
    static constexpr int NW = CT >= 8 ? 8 : CT;                       // waves
    static constexpr int NTHR = 64 * NW;
    // column tiles per wave: split BF16 pairs the re and im output tiles of the
    // same frames in one wave (each [P; M] fragment then serves both)
    static constexpr int CTW = PREC ? 2 * ((NNT + NW - 1) / NW) : (CT + NW - 1) / NW;
    static constexpr int LDC = NTP + 1;                               // staging row stride (float2)
    static constexpr int G = NTHR / TP;                               // threads per pixel for y
    static constexpr int ABYTES = TP * LDA * 4;                       // FP32 operand (k_reproj)
};

template <int NTP, int PREC, int TR>
__global__ void __launch_bounds__((RpCfg<NTP, PREC, TR>::NTHR)) k_reproj(Workspace ws) {
    static_assert(PREC == 0, "the split-BF16 reprojection is k_reproj_sb");
    using C = RpCfg<NTP, PREC, TR>;
    constexpr int IMO = C::IMO, LDA = C::LDA, LDC = C::LDC;
    constexpr int NTHR = C::NTHR, CTW = C::CTW, G = C::G, TP = C::TP, NRT = C::NRT;
    static_assert(TP % 16 == 0 && NTHR % TP == 0, "tile of whole MFMA row tiles");
    static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "y split within a row of 16 lanes");
    constexpr int TPT = NTP / G;                // frames per thread
    static_assert(NTP % G == 0, "frames split evenly over a pixel's threads");
    static_assert(C::ABYTES >= TP * LDC * 8, "the operand buffer stages the packet tile");
    __shared__ __attribute__((aligned(16))) unsigned char abuf[C::ABYTES];
    __shared__ double2 vrs[RMAX * NTP];         // V_r, [j][t]
    __shared__ float wd[TP], wsum[TP];
    __shared__ float pdsh[C::NW * TP];
    float* A = reinterpret_cast<float*>(abuf);                          // [p][LDA]
    float2* craw = reinterpret_cast<float2*>(abuf);                     // staging only: [p][LDC]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    // XCD-aware order: the grid is a multiple of 8 and block b runs on XCD b % 8
    const int per = gridDim.x >> 3;
    const int tix = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tix >= ws.ntiles) return;
    const TileDesc td = ws.tiles[tix];
    const PacketDesc pk = ws.pkts[td.pkt];
    const int nt = pk.nt, nx = pk.nx;
    const long npix = (long)pk.ny * pk.nx;
    const int npx = td.x1 - td.x0 + 1;
    // tile pixel p = row (p / TW) of the tile, column x0 + p % TW; MFMA row tile
    // a is tile row a
    static_assert(TW == 16, "one MFMA row tile per tile row");
    auto in_tile = [&](int p) { return (p / TW) < td.nrow && (p % TW) < npx; };
    auto pix_off = [&](int p) { return (long)(td.y + p / TW) * nx + td.x0 + p % TW; };
    // pixel pp of the tile is handled by the G consecutive lanes part = 0..G-1,
    // frames t = part + G i
    const int pp = tid / G, part = tid % G;

    auto put = [&](int p, int c, float re, float im) {
        A[p * LDA + c] = re;
        A[p * LDA + IMO + c] = im;
    };
    // output column tile of accumulator m: consecutive tiles per wave
    auto ct_of = [&](int m) -> int { return wave * CTW + m; };
    auto ct_ok = [&](int m) -> bool { return ct_of(m) < C::CT; };
    auto window = [&](const SubsetDesc& sd, int p) -> double {
        const int y = td.y + p / TW, x = td.x0 + p % TW;
        if (!in_tile(p) || y < sd.y0 || y > sd.y1 || x < sd.x0 || x > sd.x1) return 0.0;
        return sd.flat ? 1.0 : ws.wtab[sd.wy_off + y - sd.y0] * ws.wtab[sd.wx_off + x - sd.x0];
    };

    // the packet tile s(pixel, t): coalesced loads staged through LDS into registers
    for (int e = tid; e < TP * NTP; e += NTHR) {
        const int p = e % TP, t = e / TP;
        float2 c = make_float2(0.f, 0.f);
        if (in_tile(p) && t < nt) c = pk.iq[(long)t * npix + pix_off(p)];
        craw[p * LDC + t] = c;
    }
    __syncthreads();
    float2 sreg[TPT];
#pragma unroll
    for (int i = 0; i < TPT; ++i) sreg[i] = craw[pp * LDC + part + G * i];
    __syncthreads();
    {   // operand padding (K beyond the data) stays zero for every subset
        uint32_t* z = reinterpret_cast<uint32_t*>(abuf);
        for (int e = tid; e < C::ABYTES / 4; e += NTHR) z[e] = 0u;
    }
    floatx4 iq_acc[NRT][CTW];
    float pd_acc[NRT * 4];
#pragma unroll
    for (int a = 0; a < NRT; ++a)
#pragma unroll
        for (int m = 0; m < CTW; ++m) iq_acc[a][m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NRT * 4; ++i) pd_acc[i] = 0.f;

    // V_r of the next covering subset is loaded into registers while the
    // current one is processed (element e = tid + NTHR i of [t][j]).
    constexpr int VPT = (NTP * RMAX + NTHR - 1) / NTHR;
    double2 vnext[VPT];
    auto vload = [&](int ci) {
        const int s = ws.cover[td.cov_off + ci];
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + NTHR * i;
            vnext[i] = e < NTP * RMAX ? ws.vr64[(long)s * NTP * RMAX + e] : make_double2(0.0, 0.0);
        }
    };
    if (td.cov_cnt > 0) vload(0);

    for (int ci = 0; ci < td.cov_cnt; ++ci) {
        const int s = ws.cover[td.cov_off + ci];
        const SubsetDesc sd = ws.sub[s];
        const int r = ws.rank[s];
        const float alpha = (float)ws.alpha[s];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + NTHR * i;
            if (e < NTP * RMAX) vrs[(e % RMAX) * NTP + e / RMAX] = vnext[i];
        }
        if (tid < TP) wd[tid] = (float)window(sd, tid);
        if (ci + 1 < td.cov_cnt) vload(ci + 1);
        __syncthreads();
        // y = s V_r (FP64 partial sums over this thread's frames, then reduced over
        // the pixel's G lanes; every lane ends with the full sum), rounded to FP32
        float2 y[RMAX];
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            double yr = 0.0, yi = 0.0;
            if (j < r) {
#pragma unroll
                for (int i = 0; i < TPT; ++i) {
                    const float2 c = sreg[i];
                    const double2 v = vrs[j * NTP + part + G * i];
                    yr = fma((double)c.x, v.x, fma(-(double)c.y, v.y, yr));
                    yi = fma((double)c.x, v.y, fma((double)c.y, v.x, yi));
                }
#pragma unroll
                for (int m = G >> 1; m >= 1; m >>= 1) {
                    yr += __shfl_xor(yr, m, 64);
                    yi += __shfl_xor(yi, m, 64);
                }
            }
            y[j] = make_float2((float)yr, (float)yi);
        }
        // operand row: [c' | y] with c' = s - y V_r^H in FP64 (frames beyond nt are zero)
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const int t = part + G * i;
            double re = 0.0, im = 0.0;
            if (t < nt) {
                re = (double)sreg[i].x;
                im = (double)sreg[i].y;
#pragma unroll
                for (int j = 0; j < RMAX; ++j) {
                    if (j < r) {
                        const double2 v = vrs[j * NTP + t];
                        re -= (double)y[j].x * v.x + (double)y[j].y * v.y;
                        im -= (double)y[j].y * v.x - (double)y[j].x * v.y;
                    }
                }
            }
            put(pp, t, (float)re, (float)im);
        }
        for (int j = part; j < REXT; j += G) {
            float2 yj = make_float2(0.f, 0.f);
#pragma unroll
            for (int jj = 0; jj < RMAX; ++jj)
                if (jj == j && jj < r) yj = y[jj];
            put(pp, NTP + j, yj.x, yj.y);
        }
        __syncthreads();
        floatx4 acc[NRT][CTW];
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) acc[a][m] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float* Br = ws.breal + (long)s * (2 * C::NTE) * (2 * NTP);
#pragma unroll 4
        for (int k0 = 0; k0 < 2 * C::NTE; k0 += 4) {
            const int kk = k0 + g;
            const int acol = kk < C::NTE ? kk : IMO + kk - C::NTE;
            float av[NRT];
#pragma unroll
            for (int a = 0; a < NRT; ++a) av[a] = A[(16 * a + col) * LDA + acol];
            const float* brow = Br + (long)kk * (2 * NTP);
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                const int ct = wave * CTW + m;
                if (ct < C::CT) {
                    const float b = brow[ct * 16 + col];
#pragma unroll
                    for (int a = 0; a < NRT; ++a)
                        acc[a][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], b, acc[a][m], 0, 0, 0);
                }
            }
        }
        // epilogue: output element (pixel 16 a + 4 g + i, column ct * 16 + col)
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                if (ct_ok(m)) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float w = wd[16 * a + 4 * g + i];
                        const float v = acc[a][m][i];
                        pd_acc[a * 4 + i] += alpha * w * w * v * v;
                        iq_acc[a][m][i] += w * v;
                    }
                }
            }
    }
    // PD: reduce over the 16 lanes that share pixel rows, then over waves
#pragma unroll
    for (int i = 0; i < NRT * 4; ++i) {
        float v = pd_acc[i];
        for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
        pd_acc[i] = v;
    }
    __syncthreads();
    if (col == 0) {
#pragma unroll
        for (int i = 0; i < NRT * 4; ++i) pdsh[wave * TP + (i >> 2) * 16 + 4 * g + (i & 3)] = pd_acc[i];
    }
    if (tid < TP) {
        double ws_ = 0.0;
        for (int ci = 0; ci < td.cov_cnt; ++ci) ws_ += window(ws.sub[ws.cover[td.cov_off + ci]], tid);
        wsum[tid] = (float)ws_;
    }
    __syncthreads();
    if (tid < TP && in_tile(tid)) {
        const int p = tid;
        float pdv = 0.f;
        for (int w = 0; w < C::NW; ++w) pdv += pdsh[w * TP + p];
        if (pk.pd_mode == 2) {
            double comp = 0.0;
            for (int ci = 0; ci < td.cov_cnt; ++ci) {
                const int s = ws.cover[td.cov_off + ci];
                const double w = window(ws.sub[s], p);
                comp += ws.alpha[s] * w * w;
            }
            pdv = comp > 0.0 ? (float)((double)pdv / comp) : 0.f;
        }
        pk.pd[pix_off(p)] = pdv;
    }
    if (pk.iq_out) {
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                const int ct = ct_of(m);
                if (ct_ok(m)) {
                    const int n = ct * 16 + col;
                    const int part_ = n >= NTP, t = n - part_ * NTP;
                    if (t < nt) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int p = 16 * a + 4 * g + i;
                            if (in_tile(p)) {
                                const float w = wsum[p];
                                pk.iq_out[2 * ((long)t * npix + pix_off(p)) + part_] = w > 0.f ? iq_acc[a][m][i] / w : 0.f;
                            }
                        }
                    }
                }
            }
    }
}

// Producer/consumer form of the same reprojection. Waves 0-3 (consumers) run
// the MFMAs and the PD / IQ epilogue of covering subset d while waves 4-7
// (producers) form the operand rows [c' | y] of subset d + 1 in registers, so
// the FP64 VALU work and the matrix cores overlap on every SIMD. Two barriers
// per subset: producers write the operand (and the next V_r, window weights)
// between them, consumers read it after the second. Producer lane layout:
// pixel pt / G, frames part * TPT .. part * TPT + TPT - 1 (contiguous, so the
// operand rows are written with 16-byte stores).
template <int NTP, int PREC, int TR>
struct RpPcCfg {
    static constexpr int TP = TR * TW;
    static constexpr int NRT = TP / 16;
    static constexpr int NTE = NTP + REXT;
    static constexpr int IMO = (NTE % 32 == 16) ? NTE : NTE + 16;
    static constexpr int LDA = 2 * IMO + 4;                         // 16-byte aligned rows
    static constexpr int CT = (2 * NTP) / 16;
    static constexpr int NCW = 4, NPW = 4;                          // consumer, producer waves
    static constexpr int NTHR = 64 * (NCW + NPW);
    static constexpr int PTHR = 64 * NPW;
    static constexpr int CTW = (CT + NCW - 1) / NCW;
    static constexpr int G = PTHR / TP;                             // producer lanes per pixel
    static constexpr int TPT = NTP / G;                             // frames per producer lane
    static constexpr int YPT = (REXT + G - 1) / G;                  // y columns per producer lane
    static constexpr int LDC = NTP + 1;
    static constexpr int VPT = (NTP * RMAX + PTHR - 1) / PTHR;      // V_r elements per producer lane
    static constexpr int ABYTES = TP * LDA * 4;
};

template <int NTP, int PREC, int TR>
__global__ void __launch_bounds__((RpPcCfg<NTP, PREC, TR>::NTHR)) k_reproj_pc(Workspace ws) {
    using C = RpPcCfg<NTP, PREC, TR>;
    static_assert(PREC == 0, "the split-BF16 reprojection is k_reproj_sb");
    constexpr int IMO = C::IMO, LDA = C::LDA, LDC = C::LDC;
    constexpr int NTHR = C::NTHR, CTW = C::CTW, G = C::G, TP = C::TP, NRT = C::NRT;
    constexpr int TPT = C::TPT, YPT = C::YPT, VPT = C::VPT, PTHR = C::PTHR;
    static_assert(PTHR % TP == 0 && G >= 1 && G <= 16 && (G & (G - 1)) == 0, "pixel lanes in one row");
    static_assert(NTP % G == 0 && TPT % 8 == 0, "frames per lane in whole 16-byte groups");
    static_assert(C::ABYTES >= TP * LDC * 8, "the operand buffer stages the packet tile");
    __shared__ __attribute__((aligned(16))) unsigned char abuf[C::ABYTES];
    __shared__ double2 vrs[RMAX * NTP];         // V_r of the subset the producers work on, [j][t]
    __shared__ float wd[2][TP], wsum[TP];
    __shared__ float pdsh[C::NCW * TP];
    __shared__ float2 ysh[TP * RMAX];          // tissue scores of the subset being formed
    __shared__ float2 vrs32[RMAX * NTP];       // V_r rounded to FP32, [j][t] (for the scores only)
    float* A = reinterpret_cast<float*>(abuf);
    float2* craw = reinterpret_cast<float2*>(abuf);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool producer = wave >= C::NCW;
    const int g = lane >> 4, col = lane & 15;
    const int per = gridDim.x >> 3;
    const int tix = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tix >= ws.ntiles) return;
    const TileDesc td = ws.tiles[tix];
    const PacketDesc pk = ws.pkts[td.pkt];
    const int nt = pk.nt, nx = pk.nx;
    const long npix = (long)pk.ny * pk.nx;
    const int npx = td.x1 - td.x0 + 1;
    const int ncov = td.cov_cnt;
    auto in_tile = [&](int p) { return (p / TW) < td.nrow && (p % TW) < npx; };
    auto pix_off = [&](int p) { return (long)(td.y + p / TW) * nx + td.x0 + p % TW; };
    auto window = [&](const SubsetDesc& sd, int p) -> double {
        const int y = td.y + p / TW, x = td.x0 + p % TW;
        if (!in_tile(p) || y < sd.y0 || y > sd.y1 || x < sd.x0 || x > sd.x1) return 0.0;
        return sd.flat ? 1.0 : ws.wtab[sd.wy_off + y - sd.y0] * ws.wtab[sd.wx_off + x - sd.x0];
    };
    const int pt = tid - 64 * C::NCW;           // producer thread index
    const int pp = producer ? pt / G : 0, part = producer ? pt % G : 0;

    // packet tile, staged through LDS (all threads), kept in producer registers
    for (int e = tid; e < TP * NTP; e += NTHR) {
        const int p = e % TP, t = e / TP;
        float2 c = make_float2(0.f, 0.f);
        if (in_tile(p) && t < nt) c = pk.iq[(long)t * npix + pix_off(p)];
        craw[p * LDC + t] = c;
    }
    __syncthreads();
    // One register array holds the state of either role (a wave is one or the
    // other), so the two never compete for VGPRs:
    //   producer: packet tile s (2 TPT) | next operand rows (2 TPT) | y (2 YPT) | next V_r (4 VPT)
    //   consumer: filtered IQ accumulators (4 NRT CTW) | PD accumulators (4 NRT)
    constexpr int O_OP = 2 * TPT, O_Y = 4 * TPT, O_V = 4 * TPT + 2 * YPT, NPROD = O_V + 4 * VPT;
    constexpr int O_PD = 4 * NRT * CTW, NCONS = O_PD + 4 * NRT;
    constexpr int NST = NPROD > NCONS ? NPROD : NCONS;
    float st[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) st[k] = 0.f;
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const float2 c = producer ? craw[pp * LDC + part * TPT + i] : make_float2(0.f, 0.f);
        st[2 * i] = c.x;
        st[2 * i + 1] = c.y;
    }
    __syncthreads();
    {
        uint32_t* z = reinterpret_cast<uint32_t*>(abuf);
        for (int e = tid; e < C::ABYTES / 4; e += NTHR) z[e] = 0u;
    }
    auto sx = [&](int i) { return st[2 * i]; };
    auto sy = [&](int i) { return st[2 * i + 1]; };
    // operand words: (re, im) of frame i
    auto dset = [&](int k, double v) {
        const long long b = __double_as_longlong(v);
        st[k] = __uint_as_float((uint32_t)(b & 0xffffffff));
        st[k + 1] = __uint_as_float((uint32_t)(b >> 32));
    };
    auto dget = [&](int k) -> double {
        return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(st[k + 1]) << 32) |
                                                __float_as_uint(st[k])));
    };
    auto vload = [&](int ci) {
        const int s = ws.cover[td.cov_off + ci];
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = pt + PTHR * i;
            const double2 v = e < NTP * RMAX ? ws.vr64[(long)s * NTP * RMAX + e] : make_double2(0.0, 0.0);
            dset(O_V + 4 * i, v.x);
            dset(O_V + 4 * i + 2, v.y);
        }
    };
    auto vstore = [&]() {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = pt + PTHR * i;
            if (e < NTP * RMAX) {
                const double2 v = make_double2(dget(O_V + 4 * i), dget(O_V + 4 * i + 2));
                vrs[(e % RMAX) * NTP + e / RMAX] = v;
                vrs32[(e % RMAX) * NTP + e / RMAX] = make_float2((float)v.x, (float)v.y);
            }
        }
    };
    // operand rows of covering subset ci from vrs (producers). The tissue scores
    // y_j (one per pixel) go through ysh so that the loops over j stay rolled.
    auto form = [&](int ci) {
        const int r = ws.rank[ws.cover[td.cov_off + ci]];
#pragma unroll 1
        for (int j = 0; j < r; ++j) {
            // FP32 scores suffice: c' below is formed in FP64 from the rounded y,
            // so C' + Y V_r^H = C holds exactly whatever y is
            float yr = 0.f, yi = 0.f;
#pragma unroll
            for (int i = 0; i < TPT; ++i) {
                const float2 v = vrs32[j * NTP + part * TPT + i];
                yr = fmaf(sx(i), v.x, fmaf(-sy(i), v.y, yr));
                yi = fmaf(sx(i), v.y, fmaf(sy(i), v.x, yi));
            }
#pragma unroll
            for (int m = G >> 1; m >= 1; m >>= 1) {
                yr += __shfl_xor(yr, m, 64);
                yi += __shfl_xor(yi, m, 64);
            }
            if (part == 0) ysh[pp * RMAX + j] = make_float2(yr, yi);
        }
        // ysh is written and read by the lanes of one pixel, all in this wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const int t = part * TPT + i;
            double re = 0.0, im = 0.0;
            if (t < nt) {
                re = (double)sx(i);
                im = (double)sy(i);
#pragma unroll 1
                for (int j = 0; j < r; ++j) {
                    const float2 y = ysh[pp * RMAX + j];
                    const double2 v = vrs[j * NTP + t];
                    re -= (double)y.x * v.x + (double)y.y * v.y;
                    im -= (double)y.y * v.x - (double)y.x * v.y;
                }
            }
            st[O_OP + 2 * i] = (float)re;
            st[O_OP + 2 * i + 1] = (float)im;
        }
#pragma unroll
        for (int m = 0; m < YPT; ++m) {
            const int j = part * YPT + m;
            const float2 yj = (j < r) ? ysh[pp * RMAX + j] : make_float2(0.f, 0.f);
            st[O_Y + 2 * m] = yj.x;
            st[O_Y + 2 * m + 1] = yj.y;
        }
    };
    auto write_operand = [&]() {
        float* row = A + pp * LDA + part * TPT;
#pragma unroll
        for (int q = 0; q < TPT / 4; ++q) {
            const int f0 = O_OP + 8 * q;
            *reinterpret_cast<float4*>(row + 4 * q) = make_float4(st[f0], st[f0 + 2], st[f0 + 4], st[f0 + 6]);
            *reinterpret_cast<float4*>(row + IMO + 4 * q) = make_float4(st[f0 + 1], st[f0 + 3], st[f0 + 5], st[f0 + 7]);
        }
#pragma unroll
        for (int m = 0; m < YPT; ++m) {
            const int j = part * YPT + m;
            if (j < REXT) {
                A[pp * LDA + NTP + j] = st[O_Y + 2 * m];
                A[pp * LDA + IMO + NTP + j] = st[O_Y + 2 * m + 1];
            }
        }
    };
    // consumer accumulators live in st (zeroed above): iq (a, m, i) at 4 (a CTW + m) + i, pd at O_PD

    if (producer && ncov > 0) { vload(0); vstore(); }
    __syncthreads();
    if (producer && ncov > 0) {
        form(0);
        if (ncov > 1) vload(1);
    }
    for (int ci = 0; ci < ncov; ++ci) {
        const int s = ws.cover[td.cov_off + ci];
        __syncthreads();                               // the operand buffer is free
        if (producer) {
            write_operand();
            if (pt < TP) wd[ci & 1][pt] = (float)window(ws.sub[s], pt);
            if (ci + 1 < ncov) vstore();
        }
        __syncthreads();                               // operand of subset ci and V_r of ci + 1 ready
        if (producer) {
            if (ci + 1 < ncov) {
                if (ci + 2 < ncov) vload(ci + 2);
                form(ci + 1);
            }
            continue;
        }
        const float alpha = (float)ws.alpha[s];
        floatx4 acc[NRT][CTW];
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) acc[a][m] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float* Br = ws.breal + (long)s * (2 * C::NTE) * (2 * NTP);
#pragma unroll 2
        for (int k0 = 0; k0 < 2 * C::NTE; k0 += 4) {
            const int kk = k0 + g;
            const int acol = kk < C::NTE ? kk : IMO + kk - C::NTE;
            const float* brow = Br + (long)kk * (2 * NTP);
            float bv[CTW];
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                const int ct = wave * CTW + m;
                bv[m] = ct < C::CT ? brow[ct * 16 + col] : 0.f;
            }
#pragma unroll
            for (int a = 0; a < NRT; ++a) {
                const float av = A[(16 * a + col) * LDA + acol];
#pragma unroll
                for (int m = 0; m < CTW; ++m)
                    if (wave * CTW + m < C::CT)
                        acc[a][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[m], acc[a][m], 0, 0, 0);
            }
        }
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                if (wave * CTW + m < C::CT) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float w = wd[ci & 1][16 * a + 4 * g + i];
                        const float v = acc[a][m][i];
                        st[O_PD + a * 4 + i] += alpha * w * w * v * v;
                        st[4 * (a * CTW + m) + i] += w * v;
                    }
                }
            }
    }
    // PD: reduce over the 16 lanes that share pixel rows, then over consumer waves
    if (!producer) {
#pragma unroll
        for (int i = 0; i < NRT * 4; ++i) {
            float v = st[O_PD + i];
            for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
            st[O_PD + i] = v;
        }
    }
    __syncthreads();
    if (!producer && col == 0) {
#pragma unroll
        for (int i = 0; i < NRT * 4; ++i) pdsh[wave * TP + (i >> 2) * 16 + 4 * g + (i & 3)] = st[O_PD + i];
    }
    if (producer && pt < TP) {
        double ws_ = 0.0;
        for (int ci = 0; ci < ncov; ++ci) ws_ += window(ws.sub[ws.cover[td.cov_off + ci]], pt);
        wsum[pt] = (float)ws_;
    }
    __syncthreads();
    if (tid < TP && in_tile(tid)) {
        const int p = tid;
        float pdv = 0.f;
        for (int w = 0; w < C::NCW; ++w) pdv += pdsh[w * TP + p];
        if (pk.pd_mode == 2) {
            double comp = 0.0;
            for (int ci = 0; ci < ncov; ++ci) {
                const int s = ws.cover[td.cov_off + ci];
                const double w = window(ws.sub[s], p);
                comp += ws.alpha[s] * w * w;
            }
            pdv = comp > 0.0 ? (float)((double)pdv / comp) : 0.f;
        }
        pk.pd[pix_off(p)] = pdv;
    }
    if (pk.iq_out && !producer) {
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                const int ct = wave * CTW + m;
                if (ct < C::CT) {
                    const int n = ct * 16 + col;
                    const int part_ = n >= NTP, t = n - part_ * NTP;
                    if (t < nt) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int p = 16 * a + 4 * g + i;
                            if (in_tile(p)) {
                                const float w = wsum[p];
                                pk.iq_out[2 * ((long)t * npix + pix_off(p)) + part_] =
                                    w > 0.f ? st[4 * (a * CTW + m) + i] / w : 0.f;
                            }
                        }
                    }
                }
            }
    }
}

// Split-BF16 reprojection with the tissue scores on MFMA. The packet values of
// the tile stay in registers for all covering subsets: wave w, lane (col, g)
// holds s(16 a + col, 16 ks + g + 4 e) for its K steps ks = w + NW i, every row
// tile a and e < 4 (the accumulator layout of the FP64 residual product below;
// the score product takes them as its A operand in the same frame order, and the
// GEMM operand rows store frame g + 4 e at position 4 g + e). Per subset:
//   B  partial scores y = s V_r over the wave's frames (MFMA, split BF16; any
//      y keeps s = c' + y V_r^H exact, so its precision is free)
//   C  the partials summed in a fixed order; y in its packed operand block
//   D  c' = s - y V_r^H in FP64 on the matrix cores: per 16 frames x 16 pixels,
//      c'^T = s^T + A B with A = -conj(V_r) and B = y^T in a real form that
//      interleaves (re, im) along K (2 r <= 16), starting from the same
//      registers, which already sit in the accumulator layout of that product
//   E  chat = c' P + y M and the PD / IQ epilogue, as in k_reproj;
//      V_r and the window of the next subset go to the other LDS buffers
//
// Operand layout of [P; M] (written by k_projector<NTP, 1>): four planes (Re hi,
// Re lo, Im hi, Im lo), each [output frame n][KB] with the KC rows of P (zero
// from nt up) followed by a 32-row block that holds M in a packed real form.
// With the pixel's A row [yh_re | yh_im | yl_re | yl_im] (8 each; hi and lo of
// y, zero beyond r) the block reads
//   plane 0 [Mh_re | -Mh_im | Mh_re | -Mh_im]   plane 1 [Ml_re | -Ml_im | 0 | 0]
//   plane 2 [Mh_im |  Mh_re | Mh_im |  Mh_re]   plane 3 [Ml_im |  Ml_re | 0 | 0]
// so that two MFMAs give Re(yh Mh + yl Mh + yh Ml) and two the imaginary part:
// the three products of the split for all r <= 8 tissue columns at once.

// NWV = 4 runs four waves per tile (each with twice the output columns) in
// under 80 KB of LDS, so that two work-groups share a CU and the matrix cores
// of one overlap the FP64 / VALU phases of the other; NWV = 0 takes RpCfg's.
template <int NTP, int TR, int NWV = 0>
struct RpSbCfg {
    using R = RpCfg<NTP, 1, TR>;
    static constexpr int TP = R::TP, NRT = R::NRT, NNT = R::NNT;
    static constexpr int NW = NWV > 0 ? NWV : R::NW, NTHR = 64 * NW;
    static constexpr int CTW = 2 * ((NNT + NW - 1) / NW);
    static constexpr int VB = NWV == 4 ? 1 : 2;               // V_r buffers (one keeps LDS under 80 KB)
    static constexpr int WPE = NWV == 4 ? 2 : 1;              // work-groups asked per CU
    static constexpr int KC = SbLayout<NTP>::KC, KB = SbLayout<NTP>::KB;
    static constexpr int LDK = KB + KC + 8;                   // A row: re part + M block | im part
    static constexpr int NKS = KC / 32;                       // full complex K steps
    static constexpr int QW = CTW / 2;                        // output frame tiles per wave
    static constexpr bool QFULL = NW * QW == NNT;             // every wave's tiles exist
    static constexpr int KSTEPS = NTP / 16;                   // score K blocks of 32 (frame, re/im)
    static constexpr int MKS = (KSTEPS + NW - 1) / NW;        // K blocks per wave
    static constexpr int VPT = (NTP * RMAX + NTHR - 1) / NTHR;
    static constexpr int LDV = NTP + 1;                       // V_r row stride (double2), odd
    static constexpr int YLD = 2 * RMAX + 1;                  // y row stride (floats), odd
    // the [P; M] fragments of the next K step are requested before the MFMAs of
    // the current one where the registers allow it (else they would spill)
    static constexpr bool PREF = NTP == 128 && TR == 4 && NWV == 0;
};

typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int NTP, int TR, int NWV = 0>
__global__ void __launch_bounds__((RpSbCfg<NTP, TR, NWV>::NTHR), (RpSbCfg<NTP, TR, NWV>::WPE * RpSbCfg<NTP, TR, NWV>::NTHR / 256))
k_reproj_sb(Workspace ws) {
    using C = RpSbCfg<NTP, TR, NWV>;
    constexpr int VB = C::VB;
    constexpr int LDK = C::LDK, NTHR = C::NTHR, CTW = C::CTW, QW = C::QW, KC = C::KC, KB = C::KB;
    constexpr int TP = C::TP, NRT = C::NRT, NW = C::NW, MKS = C::MKS, VPT = C::VPT, LDV = C::LDV, YLD = C::YLD;
    static_assert(QW >= 1 && CTW == 2 * QW, "re and im output tiles in pairs");
    static_assert(RMAX == 8, "the packed M block holds 8 tissue columns");
    __shared__ __attribute__((aligned(16))) uint16_t abuf[2 * TP * LDK];
    __shared__ double2 vrs[VB][RMAX * LDV];     // V_r, [j][t], double-buffered over subsets (VB = 2)
    __shared__ float ypart[NW * TP * 16];       // score partials [wave][pixel][column]
    __shared__ float ysh[TP * YLD];             // y, [pixel][re, im of column j]
    __shared__ float wd[TP], aw2[TP];           // w and alpha w^2 of the current subset
    __shared__ float wsum[TP];
    __shared__ float pdsh[NW * TP];
    uint16_t* Ah = abuf;                        // hi: [p][LDK], re at c, M block at KC, im at KB + c
    uint16_t* Al = abuf + TP * LDK;             // lo (no M block)
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, col = lane & 15;
    // XCD-aware order: the grid is a multiple of 8 and block b runs on XCD b % 8
    const int per = gridDim.x >> 3;
    const int tix = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tix >= ws.ntiles) return;
    const TileDesc td = ws.tiles[tix];
    const PacketDesc pk = ws.pkts[td.pkt];
    const int nt = pk.nt, nx = pk.nx;
    const long npix = (long)pk.ny * pk.nx;
    const int npx = td.x1 - td.x0 + 1;
    static_assert(TW == 16, "one MFMA row tile per tile row");
    auto in_tile = [&](int p) { return (p / TW) < td.nrow && (p % TW) < npx; };
    auto pix_off = [&](int p) { return (long)(td.y + p / TW) * nx + td.x0 + p % TW; };
    // output frame tiles of this wave that exist (all of them when QFULL)
    auto qok = [&](int q) { return C::QFULL || wave * QW + q < C::NNT; };

    {   // K padding, frames from nt up and the unused lo M block stay zero
        uint32_t* z = reinterpret_cast<uint32_t*>(abuf);
        for (int e = tid; e < TP * LDK; e += NTHR) z[e] = 0u;
    }
    float2 sv[MKS][NRT][4];
#pragma unroll
    for (int i = 0; i < MKS; ++i)
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ks = wave + NW * i, p = 16 * a + col, t = 16 * ks + g + 4 * e;
                sv[i][a][e] = (ks < C::KSTEPS && in_tile(p) && t < nt) ? pk.iq[(long)t * npix + pix_off(p)]
                                                                        : make_float2(0.f, 0.f);
            }

    double2 vnext[VPT];
    auto vload = [&](int s) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + NTHR * i;
            vnext[i] = e < NTP * RMAX ? ws.vr64[(long)s * NTP * RMAX + e] : make_double2(0.0, 0.0);
        }
    };
    // V_r of a subset of rank r into buffer b, zero beyond the rank and from nt
    // up (so the score and residual products need no masks)
    auto vstore = [&](int b, int r) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int e = tid + NTHR * i;
            const int j = e % RMAX, t = e / RMAX;
            if (e < NTP * RMAX) vrs[VB == 2 ? b : 0][j * LDV + t] = (j < r && t < nt) ? vnext[i] : make_double2(0.0, 0.0);
        }
    };
    // Subset data is requested ahead of use so that no chain of dependent global
    // loads sits between two barriers: the cover index two subsets ahead, and
    // rank, weight and window geometry one subset ahead.
    struct SubNext {
        int s, r, y0, y1, x0, x1, flat, wy_off, wx_off;
        double alpha;
    };
    auto sub_load = [&](int s) {
        const SubsetDesc* d = ws.sub + s;
        return SubNext{s, ws.rank[s], d->y0, d->y1, d->x0, d->x1, d->flat, d->wy_off, d->wx_off, ws.alpha[s]};
    };
    const int ncov = td.cov_cnt;
    SubNext nxt = SubNext{0, 0, 0, -1, 0, -1, 1, 0, 0, 0.0};
    int s_ahead = 0;
    if (ncov > 0) {
        const int s0 = ws.cover[td.cov_off];
        nxt = sub_load(s0);
        vload(s0);
        vstore(0, nxt.r);
        if (ncov > 1) {
            s_ahead = ws.cover[td.cov_off + 1];
            vload(s_ahead);
        }
    }
    // window sum and sum of alpha w^2 of this thread's pixel (tid < TP), FP64
    double wsum_acc = 0.0, comp_acc = 0.0;

    floatx4 iq_acc[NRT][CTW];
    float pd_acc[NRT * 4];
#pragma unroll
    for (int a = 0; a < NRT; ++a)
#pragma unroll
        for (int m = 0; m < CTW; ++m) iq_acc[a][m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NRT * 4; ++i) pd_acc[i] = 0.f;

    for (int ci = 0; ci < ncov; ++ci) {
        const int b = VB == 2 ? (ci & 1) : 0;       // V_r buffer of this subset
        const SubNext cur = nxt;
        const int s = cur.s, r = cur.r;
        const uint16_t* planes = reinterpret_cast<const uint16_t*>(ws.breal + (long)s * (2 * (NTP + REXT)) * (2 * NTP));
        if (ci + 1 < ncov) nxt = sub_load(s_ahead);
        const int s_ahead2 = ci + 2 < ncov ? ws.cover[td.cov_off + ci + 2] : 0;
        // this subset's window factors of the thread's pixel (written to LDS after D)
        double wyv = 0.0, wxv = 0.0;
        if (tid < TP) {
            const int y = td.y + tid / TW, x = td.x0 + tid % TW;
            if (in_tile(tid) && y >= cur.y0 && y <= cur.y1 && x >= cur.x0 && x <= cur.x1) {
                wyv = cur.flat ? 1.0 : ws.wtab[cur.wy_off + y - cur.y0];
                wxv = cur.flat ? 1.0 : ws.wtab[cur.wx_off + x - cur.x0];
            }
        }
        __syncthreads();            // V_r of this subset is in; the previous GEMM is done
        // ---- B: partial scores of all row tiles over this wave's K blocks
        {
            floatx4 ya[NRT];
#pragma unroll
            for (int a = 0; a < NRT; ++a) ya[a] = floatx4{0.f, 0.f, 0.f, 0.f};
            const int j = col & 7;
            const bool imc = col >= 8;
#pragma unroll
            for (int i = 0; i < MKS; ++i) {
                const int ks = wave + NW * i;
                if (ks < C::KSTEPS) {
                    // column col of the real form: Re y_j (col < 8) or Im y_j; K row
                    // (t, re) holds (Re v, Im v), (t, im) holds (-Im v, Re v)
                    u32x4 bh, bl;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double2 v = vrs[b][j * LDV + 16 * ks + g + 4 * e];
                        uint32_t h, l;
                        split_bf16x2(imc ? (float)v.y : (float)v.x, imc ? (float)v.x : -(float)v.y, h, l);
                        bh[e] = h;
                        bl[e] = l;
                    }
                    const bf16x8 xbh = __builtin_bit_cast(bf16x8, bh), xbl = __builtin_bit_cast(bf16x8, bl);
#pragma unroll
                    for (int a = 0; a < NRT; ++a) {
                        u32x4 ah, al;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            uint32_t h, l;
                            split_bf16x2(sv[i][a][e].x, sv[i][a][e].y, h, l);
                            ah[e] = h;
                            al[e] = l;
                        }
                        const bf16x8 xah = __builtin_bit_cast(bf16x8, ah), xal = __builtin_bit_cast(bf16x8, al);
                        ya[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xah, xbh, ya[a], 0, 0, 0);
                        ya[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xah, xbl, ya[a], 0, 0, 0);
                        ya[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xal, xbh, ya[a], 0, 0, 0);
                    }
                }
            }
            // element (pixel 16 a + 4 g + i, column col)
#pragma unroll
            for (int a = 0; a < NRT; ++a)
#pragma unroll
                for (int i = 0; i < 4; ++i) ypart[(wave * TP + 16 * a + 4 * g + i) * 16 + col] = ya[a][i];
        }
        __syncthreads();
        // ---- C: y(p, j) (zero from r up) and the packed M block of the operand
        for (int e = tid; e < TP * RMAX; e += NTHR) {
            const int p = e / RMAX, j = e % RMAX;
            float yr = 0.f, yi = 0.f;
            if (j < r) {
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    yr += ypart[(w * TP + p) * 16 + j];
                    yi += ypart[(w * TP + p) * 16 + 8 + j];
                }
            }
            ysh[p * YLD + 2 * j] = yr;
            ysh[p * YLD + 2 * j + 1] = yi;
            uint32_t h, l;
            split_bf16x2(yr, yi, h, l);
            uint16_t* my = Ah + p * LDK + KC;
            my[j] = (uint16_t)h;
            my[8 + j] = (uint16_t)(h >> 16);
            my[16 + j] = (uint16_t)l;
            my[24 + j] = (uint16_t)(l >> 16);
        }
        __syncthreads();
        // ---- D: c' = s - y V_r^H (FP64 MFMA), written as four frames per store.
        // Tile (frames 16 ks .. + 15) x (pixels 16 a .. + 15); lane (col, g) holds
        // frames g + 4 e of pixel col, which go to positions 4 g + e of the operand
        // row. K chunk c holds tissue columns 2 c, 2 c + 1 as
        // k = 4 c + 2 (j - 2 c) + (0: re, 1: im):
        //   Re c' = Re s + sum_k A_re B,  A_re = (-Re v, -Im v),  B = (Re y, Im y)
        //   Im c' = Im s + sum_k A_im B,  A_im = ( Im v, -Re v)
        const int nch = (r + 1) >> 1;
#pragma unroll
        for (int i = 0; i < MKS; ++i) {
            const int ks = wave + NW * i;
            if (ks < C::KSTEPS) {
                const int t0 = 16 * ks + 4 * g;
                doublex4 cre[NRT], cim[NRT];
#pragma unroll
                for (int a = 0; a < NRT; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        // converted per subset: kept out of the loop, the FP64 copy
                        // would hold 64 more registers through every phase
                        float2 sc = sv[i][a][e];
                        asm volatile("" : "+v"(sc.x), "+v"(sc.y));
                        cre[a][e] = (double)sc.x;
                        cim[a][e] = (double)sc.y;
                    }
                const bool kim = g & 1;
                for (int c = 0; c < nch; ++c) {
                    const int j = 2 * c + (g >> 1);
                    const double2 v = vrs[b][j * LDV + 16 * ks + col];
                    const double are = kim ? -v.y : -v.x;
                    const double aim = kim ? -v.x : v.y;
#pragma unroll
                    for (int a = 0; a < NRT; ++a) {
                        const double yb = (double)ysh[(16 * a + col) * YLD + 2 * j + (g & 1)];
                        cre[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(are, yb, cre[a], 0, 0, 0);
                        cim[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, yb, cim[a], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int a = 0; a < NRT; ++a) {
                    uint32_t h[4], l[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) split_bf16x2((float)cre[a][e], (float)cim[a][e], h[e], l[e]);
                    const int p = 16 * a + col;
                    // (re of frames e, e + 1) and (im of frames e, e + 1) from two split words
                    const uint2 hre = make_uint2(__builtin_amdgcn_perm(h[1], h[0], 0x05040100u),
                                                 __builtin_amdgcn_perm(h[3], h[2], 0x05040100u));
                    const uint2 him = make_uint2(__builtin_amdgcn_perm(h[1], h[0], 0x07060302u),
                                                 __builtin_amdgcn_perm(h[3], h[2], 0x07060302u));
                    const uint2 lre = make_uint2(__builtin_amdgcn_perm(l[1], l[0], 0x05040100u),
                                                 __builtin_amdgcn_perm(l[3], l[2], 0x05040100u));
                    const uint2 lim = make_uint2(__builtin_amdgcn_perm(l[1], l[0], 0x07060302u),
                                                 __builtin_amdgcn_perm(l[3], l[2], 0x07060302u));
                    *reinterpret_cast<uint2*>(Ah + p * LDK + t0) = hre;
                    *reinterpret_cast<uint2*>(Ah + p * LDK + KB + t0) = him;
                    *reinterpret_cast<uint2*>(Al + p * LDK + t0) = lre;
                    *reinterpret_cast<uint2*>(Al + p * LDK + KB + t0) = lim;
                }
            }
        }
        // [P; M] fragments of one K step, (Re hi, Re lo, Im hi, Im lo) per frame tile;
        // the first step's are requested before the barrier ahead of E
        auto bload = [&](u32x4 (&bf)[QW][4], int kq) {
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                const int nq = wave * QW + q;
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) bf[q][pl] = u32x4{0u, 0u, 0u, 0u};
                if (qok(q)) {
                    const uint16_t* src = planes + (long)(nq * 16 + col) * KB + kq;
#pragma unroll
                    for (int pl = 0; pl < 4; ++pl)
                        bf[q][pl] = *reinterpret_cast<const u32x4*>(src + (long)pl * NTP * KB);
                }
            }
        };
        u32x4 bc[QW][4];
        if constexpr (C::PREF) bload(bc, 8 * g);
        if (tid < TP) {
            const double w = wyv * wxv;
            wd[tid] = (float)w;
            aw2[tid] = (float)(cur.alpha * w * w);
            wsum_acc += w;
            comp_acc += cur.alpha * w * w;
        }
        __syncthreads();
        // the next subset's V_r goes to the other buffer (last read by the
        // previous subset), or with one buffer over this one (its B and D are
        // done; the next B starts after the loop's first barrier)
        if (ci + 1 < ncov) {
            vstore(VB == 2 ? (b ^ 1) : 0, nxt.r);
            if (ci + 2 < ncov) vload(s_ahead2);
        }
        s_ahead = s_ahead2;
        // ---- E: chat = c' P + y M; each full K step forms
        // out_re = a_re P_re - a_im P_im and out_im = a_re P_im + a_im P_re
        floatx4 acc[NRT][CTW];
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) acc[a][m] = floatx4{0.f, 0.f, 0.f, 0.f};
        u32x4 bn[QW][4];
#pragma unroll 1
        for (int kstep = 0; kstep < C::NKS; ++kstep) {
            const int kq = 32 * kstep + 8 * g;
            if constexpr (C::PREF) bload(bn, kq + 32);      // next step; after the last P step, the M block
            else bload(bc, kq);
#pragma unroll
            for (int a = 0; a < NRT; ++a) {
                const uint16_t* arow = Ah + (16 * a + col) * LDK + kq;
                const uint16_t* lrow = Al + (16 * a + col) * LDK + kq;
                const bf16x8 xrh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(arow));
                const bf16x8 xrl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(lrow));
                const bf16x8 xih = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(arow + KB));
                const bf16x8 xil = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(lrow + KB));
#pragma unroll
                for (int q = 0; q < QW; ++q) {
                    if (qok(q)) {
                        const bf16x8 prh = __builtin_bit_cast(bf16x8, bc[q][0]), prl = __builtin_bit_cast(bf16x8, bc[q][1]);
                        const bf16x8 pih = __builtin_bit_cast(bf16x8, bc[q][2]), pil = __builtin_bit_cast(bf16x8, bc[q][3]);
                        u32x4 nh = bc[q][2], nl = bc[q][3];
#pragma unroll
                        for (int e = 0; e < 4; ++e) { nh[e] ^= 0x80008000u; nl[e] ^= 0x80008000u; }
                        const bf16x8 nih = __builtin_bit_cast(bf16x8, nh), nil = __builtin_bit_cast(bf16x8, nl);
                        floatx4& ore = acc[a][2 * q];
                        floatx4& oim = acc[a][2 * q + 1];
                        ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrh, prh, ore, 0, 0, 0);
                        ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrh, prl, ore, 0, 0, 0);
                        ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrl, prh, ore, 0, 0, 0);
                        ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xih, nih, ore, 0, 0, 0);
                        ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xih, nil, ore, 0, 0, 0);
                        ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xil, nih, ore, 0, 0, 0);
                        oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrh, pih, oim, 0, 0, 0);
                        oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrh, pil, oim, 0, 0, 0);
                        oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xrl, pih, oim, 0, 0, 0);
                        oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xih, prh, oim, 0, 0, 0);
                        oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xih, prl, oim, 0, 0, 0);
                        oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xil, prh, oim, 0, 0, 0);
                    }
                }
            }
            if constexpr (C::PREF) {
#pragma unroll
                for (int q = 0; q < QW; ++q)
#pragma unroll
                    for (int pl = 0; pl < 4; ++pl) bc[q][pl] = bn[q][pl];
            }
        }
        // the packed M block: two MFMAs per output tile
        if constexpr (!C::PREF) bload(bc, KC + 8 * g);
#pragma unroll
        for (int a = 0; a < NRT; ++a) {
            const bf16x8 xy =
                __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(Ah + (16 * a + col) * LDK + KC + 8 * g));
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                if (qok(q)) {
                    floatx4& ore = acc[a][2 * q];
                    floatx4& oim = acc[a][2 * q + 1];
                    ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xy, __builtin_bit_cast(bf16x8, bc[q][0]), ore, 0, 0, 0);
                    ore = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xy, __builtin_bit_cast(bf16x8, bc[q][1]), ore, 0, 0, 0);
                    oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xy, __builtin_bit_cast(bf16x8, bc[q][2]), oim, 0, 0, 0);
                    oim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xy, __builtin_bit_cast(bf16x8, bc[q][3]), oim, 0, 0, 0);
                }
            }
        }
        // epilogue: output element (pixel 16 a + 4 g + i, column tile of accumulator m)
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = 16 * a + 4 * g + i;
                const float w = wd[p], aw = aw2[p];
#pragma unroll
                for (int m = 0; m < CTW; ++m) {
                    if (qok(m >> 1)) {
                        const float v = acc[a][m][i];
                        pd_acc[a * 4 + i] = fmaf(aw, v * v, pd_acc[a * 4 + i]);
                        iq_acc[a][m][i] = fmaf(w, v, iq_acc[a][m][i]);
                    }
                }
            }
    }
    // PD: reduce over the 16 lanes that share pixel rows, then over waves
#pragma unroll
    for (int i = 0; i < NRT * 4; ++i) {
        float v = pd_acc[i];
        for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
        pd_acc[i] = v;
    }
    __syncthreads();
    if (col == 0) {
#pragma unroll
        for (int i = 0; i < NRT * 4; ++i) pdsh[wave * TP + (i >> 2) * 16 + 4 * g + (i & 3)] = pd_acc[i];
    }
    if (tid < TP) wsum[tid] = (float)wsum_acc;
    __syncthreads();
    if (tid < TP && in_tile(tid)) {
        const int p = tid;
        float pdv = 0.f;
        for (int w = 0; w < NW; ++w) pdv += pdsh[w * TP + p];
        if (pk.pd_mode == 2) pdv = comp_acc > 0.0 ? (float)((double)pdv / comp_acc) : 0.f;
        pk.pd[pix_off(p)] = pdv;
    }
    if (pk.iq_out) {
#pragma unroll
        for (int a = 0; a < NRT; ++a)
#pragma unroll
            for (int m = 0; m < CTW; ++m) {
                const int q = wave * QW + (m >> 1);
                if (qok(m >> 1)) {
                    const int part_ = m & 1, t = q * 16 + col;
                    if (t < nt) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int p = 16 * a + 4 * g + i;
                            if (in_tile(p)) {
                                const float w = wsum[p];
                                pk.iq_out[2 * ((long)t * npix + pix_off(p)) + part_] = w > 0.f ? iq_acc[a][m][i] / w : 0.f;
                            }
                        }
                    }
                }
            }
    }
}

// ------------------------------------------------------------------ launchers

template <int NTP>
static void post_dispatch(const Workspace& ws, int stage, int prec, hipStream_t st) {
    if (stage == 0) {
        if (prec == 0) hipLaunchKernelGGL((k_projector<NTP, 0>), dim3(ws.S), dim3(PjCfg<NTP>::NTHR), 0, st, ws);
        else hipLaunchKernelGGL((k_projector<NTP, 1>), dim3(ws.S), dim3(PjCfg<NTP>::NTHR), 0, st, ws);
    } else if (ws.ntiles > 0) {
        const int grid = (ws.ntiles + 7) / 8 * 8;      // multiple of 8 for the XCD mapping
        if constexpr (trows_max(NTP) >= 4) {
            if (ws.trows == 4 && ws.rvar == 1 && prec == 0) {
                hipLaunchKernelGGL((k_reproj_pc<NTP, 0, 4>), dim3(grid), dim3(RpPcCfg<NTP, 0, 4>::NTHR), 0, st, ws);
                return;
            }
            if (ws.trows == 4) {
                if (prec == 0)
                    hipLaunchKernelGGL((k_reproj<NTP, 0, 4>), dim3(grid), dim3(RpCfg<NTP, 0, 4>::NTHR), 0, st, ws);
                else
                    hipLaunchKernelGGL((k_reproj_sb<NTP, 4>), dim3(grid), dim3(RpSbCfg<NTP, 4>::NTHR), 0, st, ws);
                return;
            }
        }
        if (prec == 0)
            hipLaunchKernelGGL((k_reproj<NTP, 0, 2>), dim3(grid), dim3(RpCfg<NTP, 0, 2>::NTHR), 0, st, ws);
        else if constexpr (NTP == 128)
            hipLaunchKernelGGL((k_reproj_sb<NTP, 2, 4>), dim3(grid), dim3(RpSbCfg<NTP, 2, 4>::NTHR), 0, st, ws);
        else
            hipLaunchKernelGGL((k_reproj_sb<NTP, 2>), dim3(grid), dim3(RpSbCfg<NTP, 2>::NTHR), 0, st, ws);
    }
}

static hipError_t post_stage(const Workspace& ws, int stage, int prec, hipStream_t st) {
    switch (ws.ntp) {
        case 32: post_dispatch<32>(ws, stage, prec, st); break;
        case 64: post_dispatch<64>(ws, stage, prec, st); break;
        case 96: post_dispatch<96>(ws, stage, prec, st); break;
        case 128: post_dispatch<128>(ws, stage, prec, st); break;
        case 160: post_dispatch<160>(ws, stage, prec, st); break;
        case 208: post_dispatch<208>(ws, stage, prec, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rules(const Workspace& ws, const RuleParams& rp, hipStream_t st) {
    hipLaunchKernelGGL(k_rules, dim3(ws.S), dim3(64), 0, st, ws, rp);
    return hipGetLastError();
}

hipError_t launch_projector(const Workspace& ws, int precision, hipStream_t st) {
    return post_stage(ws, 0, precision, st);
}
hipError_t launch_reproj(const Workspace& ws, int precision, hipStream_t st) {
    return post_stage(ws, 1, precision, st);
}

// ------------------------------------------------------------------ diagnostics
// Copy per-subset results of subsets [first, first+count) of a packet out to the
// caller's diagnostic buffers (any pointer may be null). Eigenvectors are
// returned in the original basis: V = Q W = H_0 .. H_{r-1} W.
__global__ void __launch_bounds__(256) k_export(Workspace ws, int first, int nt, double* eigvals, float* weights,
                                               int* k, int* sweeps, int* flags, double* alpha, int* rank,
                                               double2* eigvecs, double* curve, double* mlp_gate) {
    const int d = blockIdx.x, s = first + d, tid = threadIdx.x, ntp = ws.ntp;
    for (int i = tid; i < nt; i += 256) {
        if (eigvals) eigvals[(long)d * nt + i] = ws.lam[(long)s * ntp + i];
        if (weights) weights[(long)d * nt + i] = (float)ws.wts[(long)s * ntp + i];
        if (curve) curve[(long)d * nt + i] = ws.curve[(long)s * ntp + i];
    }
    if (tid == 0) {
        if (k) k[d] = ws.kcut[s];
        if (sweeps) sweeps[d] = ws.sweeps[s];
        if (flags) flags[d] = ws.flags[s];
        if (alpha) alpha[d] = ws.alpha[s];
        if (rank) rank[d] = ws.rank[s];
        if (mlp_gate) mlp_gate[d] = ws.curve[(long)s * ntp];
    }
    if (!eigvecs) return;
    const int r = ws.rank[s];
    const double2* W = ws.bmat + (long)s * ntp * ntp;       // column-major
    for (int j = tid; j < nt; j += 256) {
        // column j, one thread; reflectors applied right to left, in place
        double2* out = eigvecs + (long)d * nt * nt + j;
        for (int t = 0; t < nt; ++t) out[(long)t * nt] = W[(long)j * ntp + t];
        for (int h = r - 1; h >= 0; --h) {
            const double tau = ws.htau[(long)s * RMAX + h];
            const double2* v = ws.hv + ((long)s * RMAX + h) * ntp;
            double2 dot = make_double2(0.0, 0.0);
            for (int t = h; t < nt; ++t) dot = cadd(dot, cmulc(v[t], out[(long)t * nt]));
            for (int t = h; t < nt; ++t) out[(long)t * nt] = csub(out[(long)t * nt], cscale(cmul(v[t], dot), tau));
        }
    }
}

__global__ void __launch_bounds__(256) k_export_cov(Workspace ws, int first, int nt, double2* cov) {
    const int d = blockIdx.x, s = first + d, ntp = ws.ntp;
    for (int e = threadIdx.x; e < nt * nt; e += 256) {
        const int t = e / nt, u = e % nt;
        cov[(long)d * nt * nt + e] = ws.pmat[(long)s * ntp * ntp + (long)t * ntp + u];
    }
}

__global__ void k_flags_or(Workspace ws, int* sticky) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < ws.S; s += gridDim.x * blockDim.x) {
        const int f = ws.flags[s];
        if (f) atomicOr(sticky, f);
    }
}

hipError_t launch_export(const Workspace& ws, int first, int count, int nt, double* eigvals, float* weights,
                         int* k, int* sweeps, int* flags, double* alpha, int* rank, double2* eigvecs,
                         double* curve, double* mlp_gate, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export, dim3(count), dim3(256), 0, st, ws, first, nt, eigvals, weights, k, sweeps,
                       flags, alpha, rank, eigvecs, curve, mlp_gate);
    return hipGetLastError();
}

hipError_t launch_export_cov(const Workspace& ws, int first, int count, int nt, double2* cov, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_cov, dim3(count), dim3(256), 0, st, ws, first, nt, cov);
    return hipGetLastError();
}

hipError_t launch_flags_or(const Workspace& ws, int* sticky, hipStream_t st) {
    hipLaunchKernelGGL(k_flags_or, dim3(1), dim3(256), 0, st, ws, sticky);
    return hipGetLastError();
}

}  // namespace lcf
