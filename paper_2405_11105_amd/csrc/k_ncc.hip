// Thresholding method 4 (Eq. 8): the cut k minimises the normalised
// cross-correlation of the tissue image I_T(k) = sum_{i=k-fn+1..k} |u_i| and
// the blood image I_B(k) = sum_{i=k+1..k+fn} |u_i| built from the left singular
// vectors u_i = C_w v_i / sigma_i of the windowed subset (C_w V = U D, so
// sigma_i = sqrt(lambda_i)), fn = 5. Method 5 is the sigmoid of Eq. 9 centred
// on that k (the rules kernel applies either shape).
//
// For every 1-based k in [fn, Nt - fn] the curve needs three sums over the
// subset's box pixels: sum I_T I_B, sum I_T^2 and sum I_B^2. Work items are the
// split-K chunks of the Gram passes; each writes those 3 x ntp sums of its
// pixels as FP64 partials, which the rules kernel adds in chunk order.
//
// The scores z_i(p) = sum_t s(p, t) v_i(t) / sigma_i are formed in FP64 from
// the FP32 packet values (exact in FP64) and the FP64 eigenvectors in the
// original basis, V = Q W; the window enters as the factor w_p of |z_i(p)|.
#include "lcf_internal.h"
#include "lcf_kernels.h"

namespace lcf {

// V / sigma in the original basis, frame-major: vs[s][t][i] = v_i(t) / sigma_i
// (0 where sigma_i = 0 or i >= nt), written over the projector buffer, which
// is free between the assembly and the projector. W (column-major in bmat) is
// taken through the r reflectors right to left, one column per thread.
__global__ void __launch_bounds__(256) k_ncc_basis(Workspace ws) {
    const int s = blockIdx.x, ntp = ws.ntp, nt = ws.sub[s].nt, r = ws.rank[s];
    const double2* W = ws.bmat + (long)s * ntp * ntp;
    double2* vs = ws.pmat + (long)s * ntp * ntp;
    const double* lam = ws.lam + (long)s * ntp;
    for (int j = threadIdx.x; j < ntp; j += blockDim.x) {
        const double l = j < nt ? lam[j] : 0.0;
        const double inv = l > 0.0 ? 1.0 / sqrt(l) : 0.0;
        if (inv == 0.0) {
            for (int t = 0; t < ntp; ++t) vs[(long)t * ntp + j] = make_double2(0.0, 0.0);
            continue;
        }
        for (int t = 0; t < ntp; ++t) vs[(long)t * ntp + j] = t < nt ? W[(long)j * ntp + t] : make_double2(0.0, 0.0);
        for (int h = r - 1; h >= 0; --h) {
            const double tau = ws.htau[(long)s * RMAX + h];
            const double2* v = ws.hv + ((long)s * RMAX + h) * ntp;
            double2 dot = make_double2(0.0, 0.0);
            for (int t = h; t < nt; ++t) dot = cadd(dot, cmulc(v[t], vs[(long)t * ntp + j]));
            for (int t = h; t < nt; ++t) vs[(long)t * ntp + j] = csub(vs[(long)t * ntp + j], cscale(cmul(v[t], dot), tau));
        }
        for (int t = 0; t < nt; ++t) vs[(long)t * ntp + j] = cscale(vs[(long)t * ntp + j], inv);
    }
}

constexpr int NCC_FN = 5;
constexpr int NCC_PB = 64;     // pixels per LDS batch (one per lane)
constexpr int NCC_NW = 8;      // waves per work-group
constexpr int NCC_TB = 8;      // frames of V / sigma staged per step

template <int NTP>
struct NccCfg {
    static constexpr int NC = NTP / NCC_NW;              // components per wave
    static constexpr int APAD = NCC_PB + 1;              // padded row of |z| (bank spread)
    static constexpr int SBYTES = NTP * NCC_PB * 8;      // raw packet values, float2 [t][p]
    static constexpr int ABYTES = NTP * APAD * 8;        // |z|, double [i][p]
    static constexpr int UBYTES = SBYTES > ABYTES ? SBYTES : ABYTES;
};

// One work-group per chunk. Per batch of 64 box pixels: (1) raw values to LDS
// (frames beyond nt and pixels beyond the chunk read as 0); (2) wave w forms
// z_i for its NC components, lane = pixel, V / sigma staged NCC_TB frames at a
// time (broadcast reads); (3) a_i(p) = w_p |z_i(p)| replaces the raw values in
// LDS; (4) thread k (0-based k - 1 for 1-based k in [fn, nt - fn]) adds the
// batch's I_T I_B, I_T^2 and I_B^2 to its registers. Zero pixels add nothing.
template <int NTP>
__global__ void __launch_bounds__(NCC_NW * 64) k_ncc_scores(Workspace ws) {
    using C = NccCfg<NTP>;
    constexpr int NTHR = NCC_NW * 64, NC = C::NC;
    __shared__ __attribute__((aligned(16))) unsigned char ubuf[C::UBYTES];
    __shared__ double2 vsb[NCC_TB * NTP];
    __shared__ double wp[NCC_PB];
    float2* sraw = (float2*)ubuf;       // [t][p]
    double* aab = (double*)ubuf;        // [i][APAD]
    const ChunkDesc ch = ws.chunks[blockIdx.x];
    const SubsetDesc sd = ws.sub[ch.s];
    const int nt = sd.nt, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double2* vs = ws.pmat + (long)ch.s * NTP * NTP;
    const double* wy = ws.wtab + sd.wy_off;
    const double* wx = ws.wtab + sd.wx_off;
    const long npix = (long)sd.ny * sd.nx;
    // curve sums of thread tid's k (1-based k = tid + 1)
    const int kk = tid + 1;
    const bool kval = kk >= NCC_FN && kk <= nt - NCC_FN;
    double s_tb = 0.0, s_tt = 0.0, s_bb = 0.0;
    for (int q0 = ch.q0; q0 < ch.q1; q0 += NCC_PB) {
        // (1) raw values, lane = pixel, waves over frames
        {
            const int q = q0 + lane;
            const bool in = q < ch.q1;
            const int y = in ? sd.y0 + q / sd.bw : sd.y0;
            const int x = in ? sd.x0 + q % sd.bw : sd.x0;
            for (int t = wave; t < NTP; t += NCC_NW) {
                float2 v = make_float2(0.f, 0.f);
                if (in && t < nt) v = sd.iq[(long)t * npix + (long)y * sd.nx + x];
                sraw[t * NCC_PB + lane] = v;
            }
            if (wave == 0) wp[lane] = in ? (sd.flat ? 1.0 : wy[y - sd.y0] * wx[x - sd.x0]) : 0.0;
        }
        // (2) scores of the wave's components
        double zr[NC], zi[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) { zr[c] = 0.0; zi[c] = 0.0; }
        for (int t0 = 0; t0 < NTP; t0 += NCC_TB) {
            __syncthreads();   // previous stage of vsb consumed; raw values written
            for (int e = tid; e < NCC_TB * NTP; e += NTHR) vsb[e] = vs[(long)t0 * NTP + e];
            __syncthreads();
#pragma unroll 2
            for (int tt = 0; tt < NCC_TB; ++tt) {
                const float2 sv = sraw[(t0 + tt) * NCC_PB + lane];
                const double sr = (double)sv.x, si = (double)sv.y;
                const double2* vrow = vsb + tt * NTP + wave * NC;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double2 v = vrow[c];
                    zr[c] = fma(sr, v.x, fma(-si, v.y, zr[c]));
                    zi[c] = fma(sr, v.y, fma(si, v.x, zi[c]));
                }
            }
        }
        __syncthreads();   // every wave done with the raw values
        // (3) a_i = w_p |z_i|
        {
            const double w = wp[lane];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                aab[(wave * NC + c) * C::APAD + lane] = w * sqrt(zr[c] * zr[c] + zi[c] * zi[c]);
        }
        __syncthreads();
        // (4) curve sums, thread = k
        if (kval) {
            for (int p = 0; p < NCC_PB; ++p) {
                double it = 0.0, ib = 0.0;
#pragma unroll
                for (int j = 0; j < NCC_FN; ++j) {
                    it += aab[(kk - NCC_FN + j) * C::APAD + p];
                    ib += aab[(kk + j) * C::APAD + p];
                }
                s_tb = fma(it, ib, s_tb);
                s_tt = fma(it, it, s_tt);
                s_bb = fma(ib, ib, s_bb);
            }
        }
        __syncthreads();   // LDS reused by the next batch
    }
    double* part = (double*)ws.partial + (long)blockIdx.x * 3 * NTP;
    if (tid < NTP) {
        part[tid] = s_tb;
        part[NTP + tid] = s_tt;
        part[2 * NTP + tid] = s_bb;
    }
}

template <int NTP>
static void ncc_dispatch(const Workspace& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_ncc_basis, dim3(ws.S), dim3(256), 0, st, ws);
    if (ws.nchunks > 0)
        hipLaunchKernelGGL((k_ncc_scores<NTP>), dim3(ws.nchunks), dim3(NCC_NW * 64), 0, st, ws);
}

hipError_t launch_ncc(const Workspace& ws, hipStream_t st) {
    switch (ws.ntp) {
        case 32: ncc_dispatch<32>(ws, st); break;
        case 64: ncc_dispatch<64>(ws, st); break;
        case 96: ncc_dispatch<96>(ws, st); break;
        case 128: ncc_dispatch<128>(ws, st); break;
        case 160: ncc_dispatch<160>(ws, st); break;
        case 208: ncc_dispatch<208>(ws, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lcf
