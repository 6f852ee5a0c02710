// Windowed temporal covariance on MFMA (Eqs 1 and 12).
//
// R_d = C_w^H C_w = sum over box pixels of w_d(x)^2 s_x^H s_x. In real form with
// a_x = Re s_x, b_x = Im s_x (rows of the Casorati matrix):
//   Re R = sum_x a_x^T a_x + b_x^T b_x        (S, symmetric)
//   Im R = sum_x a_x^T b_x - b_x^T a_x        (T, antisymmetric)
// Both are real GEMMs over an interleaved K axis (a_x, b_x, a_x+1, ...): S uses the
// operand twice, T pairs it with the row-swapped, sign-flipped copy. Only the
// upper 16x16 tiles of S and T are formed.
//
// Pass 1 (WINDOW): operand = w_d(x) * s_x, window applied on load.
// Pass 2 (DEFLATE): operand = [c'_x | y_x] with y_x = w s_x V_r (rank-r tissue
// scores) and c'_x = w s_x - y_x V_r^H formed in FP64 before rounding, so the
// fast-precision Gram only ever sees bulk-scale (blood + noise) values next to
// the separately scaled tissue columns. The extended Gram holds C'^H C',
// C'^H Y and Y^H Y.
//
// Split-K: each work-group reduces one chunk of a subset's box pixels and writes
// its partial tiles; k_gram_reduce sums the partials in chunk order in FP64, so
// results are deterministic (no atomics on data).
#include "lcf_internal.h"
#include "lcf_kernels.h"

namespace lcf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Tile order shared by both precisions and the reduction: upper tile u (i <= j,
// row-major) holds S at tau = 2u and T at tau = 2u + 1.
template <int NTP, bool DEFL, int PREC>
struct GramCfg {
    static constexpr int NTE = DEFL ? NTP + REXT : NTP;
    static constexpr int NT16 = NTE / 16;
    static constexpr int TPM = NT16 * (NT16 + 1) / 2;      // upper tiles per matrix
    static constexpr int TT = 2 * TPM;                     // S and T tiles, interleaved
    static constexpr int WAVES = TT > 60 ? 8 : 4;
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int MAXT = (TT + WAVES - 1) / WAVES;  // FP32: tiles per wave
    static constexpr int MAXP = (TPM + WAVES - 1) / WAVES; // split BF16: tile positions per wave
    // waves per SIMD asked of the register allocator: two work-groups per CU for
    // the split-BF16 pass-1 Gram up to 128 frames
    static constexpr int MIN_WAVES = (PREC == 1 && !DEFL && NTP <= 128) ? 2 * WAVES / 4 : 1;
    static constexpr int PX = NTP > 160 ? 16 : PIX;        // pixels per LDS batch
    // FP32 layout: per pixel a row [re(0..NTE) | im], odd stride
    static constexpr int IMO = (NTE % 32 == 16) ? NTE : NTE + 16;
    static constexpr int LDA = 2 * IMO + 1;
    // BF16 layout: per complex column a row of PX words (bf16 re, im), padded
    static constexpr int LDB = PX + 4;
    static constexpr int A_WORDS = PREC == 0 ? PX * LDA : 2 * NTE * LDB;
};

__device__ __forceinline__ void tile_ij(int u, int nt16, int& i, int& j) {
    int rem = u;
    i = 0;
    while (rem >= nt16 - i) { rem -= nt16 - i; ++i; }
    j = i + rem;
}

// Boxes with at least this many rows and columns are sampled in pass 1, on
// every DEC_ROWS-th row (whole rows, so that every cache line read is used).
constexpr int DEC_MIN = 8;
constexpr int DEC_ROWS = 4;

// Row fragment for the T tiles: each (re, im) word of the interleaved K axis
// becomes (-im, re), so that the product with the plain column fragment sums
// re_r im_c - im_r re_c.
__device__ __forceinline__ u32x4 swap_neg(u32x4 v) {
    u32x4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = ((v[e] >> 16) | (v[e] << 16)) ^ 0x00008000u;
    return o;
}

// Operand loads of the next batch go through global-address-space pointers:
// flat loads also count against the LDS wait counter, so every LDS wait of the
// current batch (the MFMA operand reads) would wait for them as well. A complex64
// element is loaded as one 64-bit word (re | im << 32).
typedef const uint64_t __attribute__((address_space(1)))* gptr_u64;
typedef const double __attribute__((address_space(1)))* gptr_f64;
__device__ __forceinline__ float2 c64_bits(uint64_t u, bool keep) {
    return keep ? make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)))
                : make_float2(0.f, 0.f);
}

// Split-BF16 Gram MFMAs of one batch of C::PX pixels in LDS (hi words Ah, lo
// words Al, [column][pixel] with stride LDB). K blocks of 32 = 16 pixels x
// (re, im); lane group g holds pixels 4g..4g+3. Position (i, j) of the wave:
// S from (A_i, A_j), T from (A_i swapped, A_j); acc[2m] = S, acc[2m + 1] = T.
template <class C>
__device__ __forceinline__ void gram_mfma_bf16(const uint32_t* Ah, const uint32_t* Al, const int* aoff,
                                               const int* boff, const bool* valid, floatx4* acc, int lane) {
    constexpr int LDB = C::LDB;
    const int g = lane >> 4, col = lane & 15;
#pragma unroll
    for (int kb = 0; kb < C::PX; kb += 16) {
        const int wofs = kb + 4 * g;
        int cur_a = -1;
        u32x4 ah = u32x4{0, 0, 0, 0}, al = ah, sh = ah, sl = ah;
#pragma unroll
        for (int m = 0; m < C::MAXP; ++m) {
            if (valid[m]) {
                if (aoff[m] != cur_a) {
                    cur_a = aoff[m];
                    ah = *reinterpret_cast<const u32x4*>(Ah + (cur_a + col) * LDB + wofs);
                    al = *reinterpret_cast<const u32x4*>(Al + (cur_a + col) * LDB + wofs);
                    sh = swap_neg(ah);
                    sl = swap_neg(al);
                }
                const u32x4 bh = *reinterpret_cast<const u32x4*>(Ah + (boff[m] + col) * LDB + wofs);
                const u32x4 bl = *reinterpret_cast<const u32x4*>(Al + (boff[m] + col) * LDB + wofs);
                const bf16x8 xa_h = __builtin_bit_cast(bf16x8, ah), xa_l = __builtin_bit_cast(bf16x8, al);
                const bf16x8 xs_h = __builtin_bit_cast(bf16x8, sh), xs_l = __builtin_bit_cast(bf16x8, sl);
                const bf16x8 xb_h = __builtin_bit_cast(bf16x8, bh), xb_l = __builtin_bit_cast(bf16x8, bl);
                floatx4& sa = acc[2 * m];
                floatx4& ta = acc[2 * m + 1];
                sa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa_h, xb_h, sa, 0, 0, 0);
                ta = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xs_h, xb_h, ta, 0, 0, 0);
                sa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa_h, xb_l, sa, 0, 0, 0);
                ta = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xs_h, xb_l, ta, 0, 0, 0);
                sa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa_l, xb_h, sa, 0, 0, 0);
                ta = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xs_l, xb_h, ta, 0, 0, 0);
            }
        }
    }
}

// The same at raised wave priority, for the double-buffered kernels: the other
// wave of each SIMD is forming the next batch meanwhile, and the matrix core
// should not wait for its issue slot (pass 2: 3.90 -> 3.83 ms per four-packet
// step).
template <class C>
__device__ __forceinline__ void gram_mfma_bf16_prio(const uint32_t* Ah, const uint32_t* Al, const int* aoff,
                                                    const int* boff, const bool* valid, floatx4* acc, int lane) {
    __builtin_amdgcn_s_setprio(2);
    gram_mfma_bf16<C>(Ah, Al, aoff, boff, valid, acc, lane);
    __builtin_amdgcn_s_setprio(0);
}

template <int NTP, bool DEFL, int PREC>
__global__ void __launch_bounds__((GramCfg<NTP, DEFL, PREC>::THREADS))
__attribute__((amdgpu_waves_per_eu(GramCfg<NTP, DEFL, PREC>::MIN_WAVES)))
k_gram(Workspace ws) {
    using C = GramCfg<NTP, DEFL, PREC>;
    constexpr int NTE = C::NTE, IMO = C::IMO, LDA = C::LDA, LDB = C::LDB, PIX = C::PX;
    // Split-BF16 pass 1 with eight waves double-buffers the operand: the MFMAs
    // of batch k - 1 run beside the writes of batch k (waves w and w + 4 share a
    // SIMD and take the two in opposite order), one barrier per batch.
    constexpr bool PIPE1 = !DEFL && PREC == 1 && C::WAVES == 8 && NTP <= 128;
    __shared__ __attribute__((aligned(16))) uint32_t Aw[(PIPE1 ? 2 : 1) * C::A_WORDS];
    __shared__ double2 vrs[DEFL ? RMAX * NTP : 1];     // V_r, [j][t]
    float* A = reinterpret_cast<float*>(Aw);
    uint32_t* Ah = Aw;                   // BF16 hi words [NTE][LDB] (batch being written)
    uint32_t* Al = Aw + NTE * LDB;       // BF16 lo words

    auto put = [&](int p, int c, float re, float im) {
        if (PREC == 0) {
            A[p * LDA + c] = re;
            A[p * LDA + IMO + c] = im;
        } else {
            uint32_t h, l;
            split_bf16x2(re, im, h, l);
            Ah[c * LDB + p] = h;
            Al[c * LDB + p] = l;
        }
    };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const ChunkDesc ch = ws.chunks[blockIdx.x];
    const SubsetDesc sd = ws.sub[ch.s];
    const int nt = sd.nt, nx = sd.nx;
    const long npix = (long)sd.ny * sd.nx;
    const double* wy = ws.wtab + sd.wy_off;
    const double* wx = ws.wtab + sd.wx_off;
    int r = 0;
    if (DEFL) {
        r = ws.rank[ch.s];
        for (int e = tid; e < NTP * RMAX; e += C::THREADS) {
            const int t = e / RMAX, j = e % RMAX;
            vrs[j * NTP + t] = ws.vr64[(long)ch.s * NTP * RMAX + e];
        }
    }

    // FP32: tiles tau = wave + WAVES m (round-robin). Split BF16: contiguous upper
    // tile positions u, S and T of each (row fragments shared along a tile row).
    constexpr int NACC = PREC == 0 ? C::MAXT : 2 * C::MAXP;
    constexpr int NOWN = PREC == 0 ? C::MAXT : C::MAXP;
    int aoff[NOWN], boff[NOWN];
    bool isT[NOWN], valid[NOWN];
#pragma unroll
    for (int m = 0; m < NOWN; ++m) {
        const int tau = PREC == 0 ? wave + C::WAVES * m : 2 * (wave * C::MAXP + m);
        valid[m] = tau < C::TT;
        int i, j;
        tile_ij(valid[m] ? (tau >> 1) : 0, C::NT16, i, j);
        aoff[m] = i * 16;
        boff[m] = j * 16;
        isT[m] = valid[m] && (tau & 1);
    }
    floatx4 acc[NACC];
#pragma unroll
    for (int m = 0; m < NACC; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    // FP32 pass 2 up to 128 frames: the MFMA accumulators hold one batch of PIX
    // pixels (16 K steps) and are added into FP64 sums after every batch, so FP32
    // rounding accumulates over 16 steps instead of a whole chunk (512). The bulk
    // Gram C'^H C' is what sets the FP32 path's error where a cut falls between
    // close bulk eigenvalues (the median rule at beta 1.43: 2.6e-5 -> below 1e-5).
    // Wider classes would spill the FP64 sums and keep the chunk-long accumulation.
    constexpr bool FLUSH = DEFL && PREC == 0 && NTP <= 128;
    double acc64[FLUSH ? 4 * NACC : 1];
#pragma unroll
    for (int m = 0; m < (FLUSH ? 4 * NACC : 1); ++m) acc64[m] = 0.0;

    // Operand staging is software-pipelined: the global loads of the next batch of
    // box pixels are issued before the MFMAs of the current batch. Each thread
    // owns one pixel of a batch and frames t = t0 + TSTEP i.
    //   pass 1: pixel tid % PIX, t0 = tid / PIX, TSTEP = THREADS / PIX
    //   pass 2: pixel tid / G,   t0 = tid % G,   TSTEP = G (lanes of a pixel are
    //           consecutive, so the tissue scores reduce with shuffles)
    constexpr int G = DEFL ? (C::THREADS / PIX > 16 ? 16 : C::THREADS / PIX) : 1;
    constexpr int TSTEP = DEFL ? G : C::THREADS / PIX;
    constexpr int NPT = (NTP + TSTEP - 1) / TSTEP;
    static_assert(C::THREADS % PIX == 0, "whole pixels per thread group");
    static_assert(!DEFL || NTP % G == 0, "frames split evenly over a pixel's lanes");
    const int my_p = DEFL ? tid / G : tid % PIX;
    const int my_t0 = DEFL ? tid % G : tid / PIX;
    const bool active = my_p < PIX;       // pass 2 with 16-pixel batches leaves whole waves idle
    // Loads of the next batch: every lane reads a valid address (frames beyond nt
    // clamped to frame nt - 1, pixels outside the chunk at the box origin) and the
    // mask and window product are applied when the batch is taken, so that nothing
    // waits for the loads before then. The empty asm keeps the per-frame offsets
    // from being hoisted out of the batch loop.
    uint64_t nxt[NPT];
    bool fok = false;                    // the fetched pixel lies in the chunk
    double fwy = 1.0, fwx = 1.0;         // its window factors as loaded
    // Pass 1 only has to locate the tissue subspace (any V_r keeps the pass-2
    // decomposition exact), so in split BF16 boxes of at least DEC_MIN rows and
    // columns are sampled on every DEC_ROWS-th row (the FP32 path keeps every
    // pixel: its covariance error tracks the size of C'): chunk [q0, q1) of the
    // box maps to [q0 ne / neff, q1 ne / neff) of the ne sampled pixels.
    const int bh = sd.y1 - sd.y0 + 1;
    const int dec = (!DEFL && PREC == 1 && sd.bw >= DEC_MIN && bh >= DEC_MIN) ? DEC_ROWS : 1;
    const int bwe = sd.bw;
    const long ne = (long)bwe * ((bh + dec - 1) / dec);
    const int q0 = dec == 1 ? ch.q0 : (int)((long)ch.q0 * ne / sd.neff);
    const int q1 = dec == 1 ? ch.q1 : (int)((long)ch.q1 * ne / sd.neff);
    // coordinates of this thread's pixel q = qb + my_p, advanced by PIX per batch
    int fy = (q0 + my_p) / bwe, fx = (q0 + my_p) - fy * bwe;
    const gptr_u64 giq = (gptr_u64)sd.iq;
    auto fetch = [&](int qb) {
        const int q = qb + my_p;
        const bool okp = active && q < q1;
        long pb = (long)sd.y0 * nx + sd.x0;
        fok = okp;
        if (okp) {
            pb = (long)(sd.y0 + dec * fy) * nx + sd.x0 + fx;
            if (!sd.flat) {
                fwy = ((gptr_f64)wy)[dec * fy];
                fwx = ((gptr_f64)wx)[fx];
            }
        }
        fx += PIX;
        while (fx >= bwe) { fx -= bwe; ++fy; }
        int mt = my_t0;
        asm volatile("" : "+v"(pb), "+v"(mt));
        if (active) {
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const int t = min(mt + TSTEP * i, nt - 1);
                nxt[i] = giq[(long)t * npix + pb];
            }
        }
    };
    fetch(q0);
    if constexpr (PIPE1) {
        const int nb = (q1 - q0 + PIX - 1) / PIX;
        const bool put_first = ((wave >> 2) & 1) == 0;
        for (int k = 0; k < nb + 1; ++k) {
            Ah = Aw + (k & 1) * C::A_WORDS;
            Al = Ah + NTE * LDB;
            const uint32_t* Eh = Aw + ((k & 1) ^ 1) * C::A_WORDS;    // batch k - 1
            const uint32_t* El = Eh + NTE * LDB;
            float2 cur[NPT];
#pragma unroll
            for (int i = 0; i < NPT; ++i) cur[i] = c64_bits(nxt[i], fok && my_t0 + TSTEP * i < nt);
            const double w = fok ? (sd.flat ? 1.0 : fwy * fwx) : 0.0;
            __syncthreads();                       // batch k - 1 is written, batch k - 2's MFMAs are done
            if (!put_first && k > 0) gram_mfma_bf16_prio<C>(Eh, El, aoff, boff, valid, acc, lane);
            if (k < nb) {
                const float wf = (float)w;
#pragma unroll
                for (int i = 0; i < NPT; ++i) {
                    const int t = my_t0 + TSTEP * i;
                    if (t < NTP) put(my_p, t, wf * cur[i].x, wf * cur[i].y);
                }
                if (k + 1 < nb) fetch(q0 + (k + 1) * PIX);
            }
            if (put_first && k > 0) gram_mfma_bf16_prio<C>(Eh, El, aoff, boff, valid, acc, lane);
        }
    } else
    for (int qb = q0; qb < q1; qb += PIX) {
        float2 cur[NPT];
#pragma unroll
        for (int i = 0; i < NPT; ++i) cur[i] = c64_bits(nxt[i], fok && my_t0 + TSTEP * i < nt);
        const double w = fok ? (sd.flat ? 1.0 : fwy * fwx) : 0.0;
        __syncthreads();                           // the previous batch's MFMAs are done
        // pass 2: the next batch's loads overlap the FP64 operand work as well;
        // pass 1 issues them after the (short) operand writes, reusing the registers
        if (DEFL && qb + PIX < q1) fetch(qb + PIX);
        if (!DEFL) {
            // the pass-1 Gram only locates the tissue subspace: FP32 window product
            const float wf = (float)w;
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const int t = my_t0 + TSTEP * i;
                if (t < NTP) put(my_p, t, wf * cur[i].x, wf * cur[i].y);
            }
        } else if (active) {
            // Tissue scores y = w s V_r in FP64 over this lane's frames, reduced over
            // the pixel's lanes, rounded to FP32 (any value keeps C_w = C' + Y V_r^H exact).
            float2 y[RMAX];
#pragma unroll
            for (int j = 0; j < RMAX; ++j) {
                double yr = 0.0, yi = 0.0;
                if (j < r) {
#pragma unroll
                    for (int i = 0; i < NPT; ++i) {
                        const double2 v = vrs[j * NTP + my_t0 + G * i];
                        yr = fma((double)cur[i].x, v.x, fma(-(double)cur[i].y, v.y, yr));
                        yi = fma((double)cur[i].x, v.y, fma((double)cur[i].y, v.x, yi));
                    }
#pragma unroll
                    for (int m = G >> 1; m >= 1; m >>= 1) {
                        yr += __shfl_xor(yr, m, 64);
                        yi += __shfl_xor(yi, m, 64);
                    }
                }
                y[j] = make_float2((float)(w * yr), (float)(w * yi));
            }
            // Bulk residual c' = w s - y V_r^H in FP64, rounded once.
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const int t = my_t0 + G * i;
                double re = 0.0, im = 0.0;
                if (t < nt) {
                    re = w * (double)cur[i].x;
                    im = w * (double)cur[i].y;
#pragma unroll
                    for (int j = 0; j < RMAX; ++j) {
                        if (j < r) {
                            const double2 v = vrs[j * NTP + t];
                            // y * conj(v)
                            re -= (double)y[j].x * v.x + (double)y[j].y * v.y;
                            im -= (double)y[j].y * v.x - (double)y[j].x * v.y;
                        }
                    }
                }
                put(my_p, t, (float)re, (float)im);
            }
            for (int j = my_t0; j < REXT; j += G) {
                float2 yj = make_float2(0.f, 0.f);
#pragma unroll
                for (int jj = 0; jj < RMAX; ++jj)
                    if (jj == j && jj < r) yj = y[jj];
                put(my_p, NTP + j, yj.x, yj.y);
            }
        }
        if (!DEFL && qb + PIX < q1) fetch(qb + PIX);   // in flight during the MFMAs
        __syncthreads();
        if (PREC == 0) {
            const int kk = lane >> 4, col = lane & 15;
#pragma unroll 2
            for (int kp = 0; kp < PIX; kp += 2) {
                const int p = kp + (kk >> 1), part = kk & 1;
                const float* rowp = A + p * LDA;
                const float* base = rowp + (part ? IMO : 0);
                const float* swp = part ? rowp : rowp + IMO;      // partner part for T
                const float sgn = part ? -1.f : 1.f;
#pragma unroll
                for (int m = 0; m < C::MAXT; ++m) {
                    if (valid[m]) {
                        const float a = base[aoff[m] + col];
                        const float b = isT[m] ? sgn * swp[boff[m] + col] : base[boff[m] + col];
                        acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[m], 0, 0, 0);
                    }
                }
            }
            if (FLUSH) {
#pragma unroll
                for (int m = 0; m < NACC; ++m) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc64[4 * m + e] += (double)acc[m][e];
                    acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
            }
        } else {
            gram_mfma_bf16<C>(Ah, Al, aoff, boff, valid, acc, lane);
        }
    }
#pragma unroll
    for (int m = 0; m < NACC; ++m) {
        const int tau = PREC == 0 ? wave + C::WAVES * m : 2 * (wave * C::MAXP + (m >> 1)) + (m & 1);
        if (tau < C::TT) {
            float* dst = ws.partial + ((long)blockIdx.x * C::TT + tau) * 256 + lane * 4;
            if (FLUSH) {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[m][e] = (float)acc64[4 * m + e];
            }
            *reinterpret_cast<floatx4*>(dst) = acc[m];
        }
    }
}
// Pass 2 in split BF16 (DEFLATE). Each batch of PX box pixels goes through:
//  A  coalesced loads -> raw s (FP32) and the split rows w s (LDS)
//  B  tissue scores y = (w s) V_r on MFMA, split BF16, K split over waves (any
//     y keeps C_w = C' + Y V_r^H exact, so its precision is free)
//  C  each wave sums the partial scores of its own pixels in a fixed order and
//     writes the y columns of the operand
//  D  c' = w s - y V_r^H in FP64, one lane per frame: every V_r row read from
//     LDS serves all pixels of the wave
//  E  the Gram MFMAs over [c' | y] (as in pass 1)
template <int NTP>
struct DeflCfg {
    using GC = GramCfg<NTP, true, 1>;
    static constexpr int NTE = GC::NTE, LDB = GC::LDB, PX = GC::PX;
    static constexpr int WAVES = GC::WAVES, THREADS = GC::THREADS;
    static constexpr int MT = PX / 16;                    // y row tiles
    static constexpr int KSTEPS = NTP / 16;               // K blocks of 32 over (frame, re/im)
    static constexpr int KG = WAVES / MT;                 // K groups (one partial each)
    static constexpr int MAXKS = (KSTEPS + KG - 1) / KG;
    static constexpr int NPT = 4 * MAXKS;                 // phase A values per lane (the B operand's frames)
    static constexpr int LDS_S = NTP + 1;                 // raw row stride (float2), odd
    static constexpr int FPT = (NTP + 63) / 64;           // phase D frames per lane
    static constexpr int PPW = PX / WAVES;                // phase D pixels per wave
    static_assert(PX % 16 == 0 && WAVES % MT == 0 && THREADS % PX == 0, "tiling");
    static_assert(PPW * 16 <= 128 && PPW >= 1, "phase C lanes");
};

template <int NTP>
__global__ void __launch_bounds__((DeflCfg<NTP>::THREADS)) k_gram_defl(Workspace ws) {
    using D = DeflCfg<NTP>;
    using C = typename D::GC;
    constexpr int NTE = D::NTE, LDB = D::LDB, PX = D::PX, WAVES = D::WAVES;
    // With eight waves (up to 128 frames; above, the second buffer does not fit
    // in LDS) the operand is double-buffered: the Gram MFMAs of batch k - 1 run
    // in the same phase as C and D of batch k, on every SIMD one wave doing the
    // FP64 residual while the other issues MFMAs (waves w and w + 4 share a SIMD
    // and take the two in opposite order).
    constexpr bool PIPE = WAVES == 8 && NTP <= 128;
    constexpr int BUFW = 2 * NTE * LDB;                  // words of one operand buffer (hi, lo)
    __shared__ __attribute__((aligned(16))) uint32_t Aw[(PIPE ? 2 : 1) * BUFW];
    __shared__ float2 sraw[PX * D::LDS_S];
    __shared__ double2 vrs[RMAX * NTP];                  // V_r, [j][t]
    __shared__ float ypart[D::KG * PX * 16];
    __shared__ float2 ysh[PX * RMAX];
    __shared__ double wsh[PX];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, col = lane & 15;
    const ChunkDesc ch = ws.chunks[blockIdx.x];
    const SubsetDesc sd = ws.sub[ch.s];
    const int nt = sd.nt, nx = sd.nx;
    const long npix = (long)sd.ny * sd.nx;
    const double* wy = ws.wtab + sd.wy_off;
    const double* wx = ws.wtab + sd.wx_off;
    const int r = ws.rank[ch.s];
    for (int e = tid; e < NTP * RMAX; e += D::THREADS) {
        const int t = e / RMAX, j = e % RMAX;
        vrs[j * NTP + t] = ws.vr64[(long)ch.s * NTP * RMAX + e];
    }

    // Phase B operands of this wave: row tile ymt, K steps ykg + KG i. Column n of
    // the real form: n < 8 gives Re y_n, n >= 8 gives Im y_(n-8); K row (t, re)
    // holds (Re v, Im v) and (t, im) holds (-Im v, Re v).
    const int ymt = wave % D::MT, ykg = wave / D::MT;
    u32x4 vbh[D::MAXKS], vbl[D::MAXKS];
#pragma unroll
    for (int i = 0; i < D::MAXKS; ++i) {
        const int ks = ykg + D::KG * i;
        const int j = col & 7;
        const bool imcol = col >= 8;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t = 16 * ks + 4 * g + e;
            float kr = 0.f, ki = 0.f;
            if (ks < D::KSTEPS && t < nt && j < r) {
                const float2 v = ws.vr32[((long)ch.s * NTP + t) * RMAX + j];
                kr = imcol ? v.y : v.x;
                ki = imcol ? v.x : -v.y;
            }
            uint32_t h, l;
            split_bf16x2(kr, ki, h, l);
            vbh[i][e] = h;
            vbl[i][e] = l;
        }
    }

    // Gram tile positions (contiguous upper positions, S and T of each)
    int aoff[C::MAXP], boff[C::MAXP];
    bool valid[C::MAXP];
#pragma unroll
    for (int m = 0; m < C::MAXP; ++m) {
        const int u = wave * C::MAXP + m;
        valid[m] = u < C::TPM;
        int i, j;
        tile_ij(valid[m] ? u : 0, C::NT16, i, j);
        aoff[m] = i * 16;
        boff[m] = j * 16;
    }
    floatx4 acc[2 * C::MAXP];
#pragma unroll
    for (int m = 0; m < 2 * C::MAXP; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};

    // phase A layout: lane (col, g) of wave (ymt, ykg) loads pixel 16 ymt + col at
    // the frames of its phase-B operand, 16 ks + 4 g + e for ks = ykg + KG i, so
    // that the scores take their operand from registers; the loads of the next
    // batch are in flight meanwhile
    const int my_p = 16 * ymt + col;
    // loads as in k_gram: valid addresses, mask and window product applied in phase A
    uint64_t nxt[D::NPT];
    bool fok = false;
    double fwy = 1.0, fwx = 1.0;
    const gptr_u64 giq = (gptr_u64)sd.iq;
    int fy = (ch.q0 + my_p) / sd.bw, fx = (ch.q0 + my_p) - fy * sd.bw;
    auto fetch = [&](int qb) {
        const int q = qb + my_p;
        const bool okp = q < ch.q1;
        long pb = (long)sd.y0 * nx + sd.x0;
        fok = okp;
        if (okp) {
            pb = (long)(sd.y0 + fy) * nx + sd.x0 + fx;
            if (!sd.flat) {
                fwy = ((gptr_f64)wy)[fy];
                fwx = ((gptr_f64)wx)[fx];
            }
        }
        fx += PX;
        while (fx >= sd.bw) { fx -= sd.bw; ++fy; }
        int mt = 16 * ykg + 4 * g;
        asm volatile("" : "+v"(pb), "+v"(mt));
#pragma unroll
        for (int i = 0; i < D::MAXKS; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int t = min(mt + 16 * D::KG * i + e, nt - 1);
                nxt[4 * i + e] = giq[(long)t * npix + pb];
            }
    };
    const int nb = (ch.q1 - ch.q0 + PX - 1) / PX;
    const bool cd_first = !PIPE || ((wave >> 2) & 1) == 0;
    fetch(ch.q0);
    for (int k = 0; k < nb + (PIPE ? 1 : 0); ++k) {
        const int qb = ch.q0 + k * PX;
        uint32_t* Ah = Aw + (PIPE ? (k & 1) * BUFW : 0);     // operand being formed: batch k
        uint32_t* Al = Ah + NTE * LDB;
        const uint32_t* Eh = PIPE ? Aw + ((k & 1) ^ 1) * BUFW : Ah;   // Gram of batch k - 1 (PIPE) or k
        const uint32_t* El = Eh + NTE * LDB;
        const bool work = k < nb, egram = PIPE ? k > 0 : true;
        __syncthreads();                           // the previous batch's C, D and E are done
        // ---- A: raw values to LDS for the residual (which then writes every
        // operand row below NTP), the split window products kept for B
        u32x4 xh[D::MAXKS], xl[D::MAXKS];
        if (work) {
            const double nw = fok ? (sd.flat ? 1.0 : fwy * fwx) : 0.0;
            const float wf = (float)nw;
            if (ykg == 0 && g == 0) wsh[my_p] = nw;
#pragma unroll
            for (int i = 0; i < D::MAXKS; ++i) {
                xh[i] = u32x4{0, 0, 0, 0};
                xl[i] = xh[i];
                const int ks = ykg + D::KG * i;
                if (ks < D::KSTEPS) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int t = 16 * ks + 4 * g + e;
                        const float2 c = c64_bits(nxt[4 * i + e], fok && t < nt);
                        sraw[my_p * D::LDS_S + t] = c;
                        uint32_t h, l;
                        split_bf16x2(wf * c.x, wf * c.y, h, l);
                        xh[i][e] = h;
                        xl[i][e] = l;
                    }
                }
            }
        }
        if (work && qb + PX < ch.q1) fetch(qb + PX);   // in flight until the next batch
        // ---- B: y partial of row tile ymt over this wave's K steps, from registers
        if (work) {
            floatx4 ya = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < D::MAXKS; ++i) {
                const int ks = ykg + D::KG * i;
                if (ks < D::KSTEPS) {
                    const bf16x8 ah = __builtin_bit_cast(bf16x8, xh[i]), al = __builtin_bit_cast(bf16x8, xl[i]);
                    const bf16x8 bh = __builtin_bit_cast(bf16x8, vbh[i]), bl = __builtin_bit_cast(bf16x8, vbl[i]);
                    ya = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, ya, 0, 0, 0);
                    ya = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, ya, 0, 0, 0);
                    ya = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, ya, 0, 0, 0);
                }
            }
            // element (pixel 16 ymt + 4 g + i, column col)
#pragma unroll
            for (int i = 0; i < 4; ++i) ypart[(ykg * PX + 16 * ymt + 4 * g + i) * 16 + col] = ya[i];
        }
        __syncthreads();                           // A's raw values and B's partials are in
        if (PIPE && !cd_first && egram) gram_mfma_bf16_prio<C>(Eh, El, aoff, boff, valid, acc, lane);
        // ---- C: scores of this wave's pixels (lane: pixel 16-lane group, column)
        if (work) {
#pragma unroll
            for (int h2 = 0; h2 < (D::PPW * 16 + 63) / 64; ++h2) {
                const int kp = (lane >> 4) + 4 * h2;            // pixel of the wave
                const bool on = kp < D::PPW;
                const int p = wave * D::PPW + (on ? kp : 0);
                float v = 0.f;
#pragma unroll
                for (int q = 0; q < D::KG; ++q) v += ypart[(q * PX + p) * 16 + col];
                // (Re y_j, Im y_j) meet in lane col = j after a rotate by 8 within the row
                const float vi = __shfl_xor(v, 8, 16);
                const int j = col;
                float yr = 0.f, yi = 0.f;
                if (j < RMAX && j < r) { yr = v; yi = vi; }
                if (on) {
                    if (j < RMAX) ysh[p * RMAX + j] = make_float2(yr, yi);
                    uint32_t hh, ll;
                    split_bf16x2(yr, yi, hh, ll);
                    Ah[(NTP + j) * LDB + p] = hh;      // REXT = 16 columns, zero beyond r
                    Al[(NTP + j) * LDB + p] = ll;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // ---- D: c' = w s - y V_r^H for frames lane + 64 f, pixels of the wave
            {
                double cr[D::PPW][D::FPT], ci[D::PPW][D::FPT];
                double wp[D::PPW];
#pragma unroll
                for (int kp = 0; kp < D::PPW; ++kp) {
                    const int p = wave * D::PPW + kp;
                    wp[kp] = wsh[p];
#pragma unroll
                    for (int f = 0; f < D::FPT; ++f) {
                        const int t = lane + 64 * f;
                        const float2 c = t < NTP ? sraw[p * D::LDS_S + t] : make_float2(0.f, 0.f);
                        cr[kp][f] = wp[kp] * (double)c.x;
                        ci[kp][f] = wp[kp] * (double)c.y;
                    }
                }
                for (int j = 0; j < r; ++j) {
                    double2 v[D::FPT];
#pragma unroll
                    for (int f = 0; f < D::FPT; ++f) {
                        const int t = lane + 64 * f;
                        v[f] = t < NTP ? vrs[j * NTP + t] : make_double2(0.0, 0.0);
                    }
#pragma unroll
                    for (int kp = 0; kp < D::PPW; ++kp) {
                        const float2 yk = ysh[(wave * D::PPW + kp) * RMAX + j];
                        const double yr = (double)yk.x, yi = (double)yk.y;
#pragma unroll
                        for (int f = 0; f < D::FPT; ++f) {
                            // minus y * conj(v)
                            cr[kp][f] = fma(-yr, v[f].x, fma(-yi, v[f].y, cr[kp][f]));
                            ci[kp][f] = fma(-yi, v[f].x, fma(yr, v[f].y, ci[kp][f]));
                        }
                    }
                }
                // the wave's PPW pixels are adjacent in an operand row: one store
                // of up to 16 bytes per frame (single words at stride LDB would
                // meet in a quarter of the banks)
                constexpr int VW = D::PPW % 4 == 0 ? 4 : D::PPW % 2 == 0 ? 2 : 1;
#pragma unroll
                for (int f = 0; f < D::FPT; ++f) {
                    const int t = lane + 64 * f;
                    if (t < NTP) {
                        const bool in = t < nt;
#pragma unroll
                        for (int k0 = 0; k0 < D::PPW; k0 += VW) {
                            uint32_t h[VW], l[VW];
#pragma unroll
                            for (int v = 0; v < VW; ++v)
                                split_bf16x2(in ? (float)cr[k0 + v][f] : 0.f, in ? (float)ci[k0 + v][f] : 0.f, h[v], l[v]);
                            const int o = t * LDB + wave * D::PPW + k0;
                            if constexpr (VW == 4) {
                                *reinterpret_cast<u32x4*>(Ah + o) = u32x4{h[0], h[1], h[2], h[3]};
                                *reinterpret_cast<u32x4*>(Al + o) = u32x4{l[0], l[1], l[2], l[3]};
                            } else if constexpr (VW == 2) {
                                *reinterpret_cast<uint2*>(Ah + o) = make_uint2(h[0], h[1]);
                                *reinterpret_cast<uint2*>(Al + o) = make_uint2(l[0], l[1]);
                            } else {
                                Ah[o] = h[0];
                                Al[o] = l[0];
                            }
                        }
                    }
                }
            }
        }
        if (!PIPE) __syncthreads();
        // ---- E
        if (cd_first && egram) gram_mfma_bf16_prio<C>(Eh, El, aoff, boff, valid, acc, lane);
    }
#pragma unroll
    for (int m = 0; m < 2 * C::MAXP; ++m) {
        const int tau = 2 * (wave * C::MAXP + (m >> 1)) + (m & 1);
        if (tau < C::TT) {
            float* dst = ws.partial + ((long)blockIdx.x * C::TT + tau) * 256 + lane * 4;
            *reinterpret_cast<floatx4*>(dst) = acc[m];
        }
    }
}

// Sum the chunk partials of each subset in chunk order (FP64) and expand the
// upper S/T tiles into the full Hermitian matrix out[s][NTE][NTE].
// T = double2 (pass 2: the extended Gram) or float2 (pass 1).
template <int NTE, class T>
__global__ void __launch_bounds__(256) k_gram_reduce(Workspace ws, T* out, int tt) {
    constexpr int NT16 = NTE / 16;
    const int s = blockIdx.y;
    const int u = blockIdx.x;
    int i, j;
    tile_ij(u, NT16, i, j);
    const int e = threadIdx.x;
    const int lane = e >> 2, rr = e & 3;
    const int rin = 4 * (lane >> 4) + rr, cin = lane & 15;
    if (i == j && rin > cin) return;
    const int c0 = ws.chunk_begin[s], c1 = ws.chunk_begin[s + 1];
    double sv = 0.0, tv = 0.0;
    for (int c = c0; c < c1; ++c) {
        sv += (double)ws.partial[((long)c * tt + 2 * u) * 256 + e];
        tv += (double)ws.partial[((long)c * tt + 2 * u + 1) * 256 + e];
    }
    const int row = i * 16 + rin, colx = j * 16 + cin;
    T* o = out + (long)s * NTE * NTE;
    using E = decltype(o->x);
    if (row == colx) {
        o[(long)row * NTE + colx] = T{(E)sv, (E)0};
    } else {
        o[(long)row * NTE + colx] = T{(E)sv, (E)tv};
        o[(long)colx * NTE + row] = T{(E)sv, (E)(-tv)};
    }
    if (!isfinite(sv) || !isfinite(tv)) atomicOr(&ws.flags[s], 2);
}

// ------------------------------------------------------------------ launchers

template <int NTP, bool DEFL, int PREC>
static void gram_launch(const Workspace& ws, bool reduce, hipStream_t st) {
    using C = GramCfg<NTP, DEFL, PREC>;
    if (!reduce) {
        if (DEFL && PREC == 1) hipLaunchKernelGGL((k_gram_defl<NTP>), dim3(ws.nchunks), dim3(C::THREADS), 0, st, ws);
        else hipLaunchKernelGGL((k_gram<NTP, DEFL, (DEFL ? 0 : PREC)>), dim3(ws.nchunks), dim3(C::THREADS), 0, st, ws);
    }
    else if constexpr (DEFL)
        hipLaunchKernelGGL((k_gram_reduce<C::NTE, double2>), dim3(C::TPM, ws.S), dim3(256), 0, st, ws, ws.rext, C::TT);
    else
        hipLaunchKernelGGL((k_gram_reduce<C::NTE, float2>), dim3(C::TPM, ws.S), dim3(256), 0, st, ws, ws.rwin, C::TT);
}

template <int NTP>
static hipError_t gram_dispatch(const Workspace& ws, bool defl, bool reduce, int prec, hipStream_t st) {
    if (ws.nchunks == 0) return hipSuccess;
    if (defl) {
        if (prec == 0) gram_launch<NTP, true, 0>(ws, reduce, st);
        else gram_launch<NTP, true, 1>(ws, reduce, st);
    } else {
        if (prec == 0) gram_launch<NTP, false, 0>(ws, reduce, st);
        else gram_launch<NTP, false, 1>(ws, reduce, st);
    }
    return hipGetLastError();
}

// reduce = false: the split-K Gram kernel; reduce = true: the ordered FP64 reduction.
hipError_t launch_gram(const Workspace& ws, bool defl, bool reduce, int precision, hipStream_t st) {
    switch (ws.ntp) {
        case 32: return gram_dispatch<32>(ws, defl, reduce, precision, st);
        case 64: return gram_dispatch<64>(ws, defl, reduce, precision, st);
        case 96: return gram_dispatch<96>(ws, defl, reduce, precision, st);
        case 128: return gram_dispatch<128>(ws, defl, reduce, precision, st);
        case 160: return gram_dispatch<160>(ws, defl, reduce, precision, st);
        case 208: return gram_dispatch<208>(ws, defl, reduce, precision, st);
        default: return hipErrorInvalidValue;
    }
}

int gram_tiles(int ntp, bool defl) {
    const int nte = defl ? ntp + REXT : ntp;
    const int n16 = nte / 16;
    return n16 * (n16 + 1);
}

}  // namespace lcf
