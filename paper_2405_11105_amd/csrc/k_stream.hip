// Covariance of sliding packets. When packet p + 1 holds frames [h, nt) of
// packet p followed by h new frames, every entry of R_{p+1} = C_w^H C_w (Eqs 1,
// 12) between two retained frames is an entry of R_p: R_{p+1}[i][j] =
// R_p[i + h][j + h] for i, j < nt - h. Only the h new columns (and their
// conjugate rows) are summed over the box pixels, in FP64 from the FP32 packet
// values, so no entry is ever updated by subtraction and nothing drifts. The
// FP64 covariance then stands in for both Gram passes of a packet: it is
// rounded to FP32 for the tissue basis and handed to the assembly as the
// deflated Gram with zero tissue blocks (the assembly then forms B = Q^H R Q).
#include "lcf_internal.h"
#include "lcf_kernels.h"

namespace lcf {

constexpr int SC_PB = 32;    // pixels per LDS batch
constexpr int SC_NC = 16;    // new columns per work-group (the partials' row length)

// Work-group (s, g, b): new columns j0 .. j0 + NCM - 1 (j0 = nt - h + 16 g, at most
// 16) of subset s over row band b of its box. Per batch of 32 box pixels the
// raw values of every frame sit in LDS as [pixel][frame] (the next batch is
// loaded into registers meanwhile); thread (i, half) accumulates
// sum_x w_x^2 conj(s(x, t_i)) s(x, t_j) for row i, every column of the group and
// its share of the batch's pixels; the halves are added in a fixed order and
// the band's sums go to part[s][g][b][i][16]. NCM = 8 serves hops up to 8
// with half the accumulators (more waves per SIMD).
template <int NTP, int NCM>
__global__ void __launch_bounds__(256, (NCM <= 8 && NTP <= 128) ? 4 : 1) k_cov_new(Workspace ws, double2* part, int hop, int ngroups, int nband) {
    constexpr int LDP = NTP + 1;                        // row of one pixel (float2), odd stride
    constexpr int HALVES = 256 / NTP > 0 ? 256 / NTP : 1;
    constexpr int PPH = SC_PB / HALVES;                 // pixels per half
    constexpr int LT = 256 / SC_PB;                     // frame lanes of the loader
    constexpr int TPT = NTP / LT;                       // frames loaded per thread per batch
    __shared__ float2 sr[SC_PB * LDP];
    __shared__ double w2[SC_PB];
    const int s = blockIdx.x, g = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
    const SubsetDesc sd = ws.sub[s];
    const int nt = sd.nt;
    const int j0 = nt - hop + SC_NC * g;
    const int ncol = min(NCM, nt - j0);
    const int nrow = sd.y1 - sd.y0 + 1;
    const int r0 = (int)((long)nrow * b / nband), r1 = (int)((long)nrow * (b + 1) / nband);
    const int q0 = r0 * sd.bw, q1 = r1 * sd.bw;
    const double* wy = ws.wtab + sd.wy_off;
    const double* wx = ws.wtab + sd.wx_off;
    const long npix = (long)sd.ny * sd.nx;
    // loader role: pixel lp of the batch, frames lt0 + LT k
    const int lp = tid & (SC_PB - 1), lt0 = tid / SC_PB;
    // compute role: row i, pixels [half * PPH, (half + 1) * PPH) of the batch
    const int i = tid % NTP, half = tid / NTP;
    const bool crow = half < HALVES && i < nt;
    float2 pre[TPT];
    double wpre = 0.0;
    auto fetch = [&](int qb) {
        const int q = qb + lp;
        const bool in = q < q1;
        const int y = in ? sd.y0 + q / sd.bw : sd.y0;
        const int x = in ? sd.x0 + q % sd.bw : sd.x0;
        const float2* src = sd.iq + (long)y * sd.nx + x;
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const int t = lt0 + LT * k;
            pre[k] = (in && t < nt) ? src[(long)t * npix] : make_float2(0.f, 0.f);
        }
        if (lt0 == 0) {
            const double w = in ? (sd.flat ? 1.0 : wy[y - sd.y0] * wx[x - sd.x0]) : 0.0;
            wpre = w * w;
        }
    };
    double2 acc[NCM];
#pragma unroll
    for (int c = 0; c < NCM; ++c) acc[c] = make_double2(0.0, 0.0);
    if (q0 < q1) fetch(q0);
    for (int qb = q0; qb < q1; qb += SC_PB) {
        __syncthreads();   // previous batch consumed
#pragma unroll
        for (int k = 0; k < TPT; ++k) sr[lp * LDP + lt0 + LT * k] = pre[k];
        if (lt0 == 0) w2[lp] = wpre;
        __syncthreads();
        if (qb + SC_PB < q1) fetch(qb + SC_PB);     // in flight during the products
        if (crow) {
#pragma unroll 1
            for (int p = half * PPH; p < (half + 1) * PPH; ++p) {
                const float2 a = sr[p * LDP + i];
                const double ww = w2[p];
                const double ar = (double)a.x * ww, ai = -(double)a.y * ww;   // w^2 conj(a)
                const float2* brow = sr + p * LDP + j0;
#pragma unroll
                for (int c = 0; c < NCM; ++c) {
                    if (c < ncol) {
                        const float2 bv = brow[c];
                        const double br = (double)bv.x, bi = (double)bv.y;
                        acc[c].x = fma(ar, br, fma(-ai, bi, acc[c].x));
                        acc[c].y = fma(ar, bi, fma(ai, br, acc[c].y));
                    }
                }
            }
        }
    }
    // add the halves in order through LDS (the batch buffer is free again)
    double2* red = reinterpret_cast<double2*>(sr);
    static_assert(SC_PB * LDP * sizeof(float2) >= NTP * NCM * sizeof(double2),
                  "the batch buffer holds the halves' partial sums");
    for (int hh = 1; hh < HALVES; ++hh) {
        __syncthreads();
        if (half == hh && crow) {
#pragma unroll
            for (int c = 0; c < NCM; ++c) red[i * NCM + c] = acc[c];
        }
        __syncthreads();
        if (half == 0 && crow) {
#pragma unroll
            for (int c = 0; c < NCM; ++c) {
                const double2 v = red[i * NCM + c];
                acc[c].x += v.x;
                acc[c].y += v.y;
            }
        }
    }
    if (half == 0 && i < NTP) {
        double2* o = part + ((((long)s * ngroups + g) * nband + b) * NTP + i) * SC_NC;
#pragma unroll
        for (int c = 0; c < SC_NC; ++c) o[c] = (i < nt && c < NCM) ? acc[c < NCM ? c : 0] : make_double2(0.0, 0.0);
    }
}

// Row i of R_new for subset s (thread = column j, so every access runs along a
// row): entries between retained frames copy R_old shifted by h; an entry in a
// new column j >= i is the sum of the band partials of (i, j) in band order,
// and an entry in a new row i > j is the conjugate of that sum for (j, i), so
// R_new is exactly Hermitian with a real diagonal.
template <int NTP>
__global__ void __launch_bounds__(256) k_cov_finish(Workspace ws, const double2* rold, double2* rnew,
                                                    const double2* part, int hop, int ngroups, int nband) {
    const int s = blockIdx.x, i = blockIdx.y, j = threadIdx.x;
    const int nt = ws.sub[s].nt;
    if (i >= nt || j >= nt) return;
    const long base = (long)s * NTP * NTP;
    const int nold = nt - hop;
    if (i < nold && j < nold) {
        rnew[base + (long)i * NTP + j] = rold[base + (long)(i + hop) * NTP + (j + hop)];
        return;
    }
    // (a, c) with c the new column: (i, j) itself when j >= i, else its mirror (j, i)
    const bool mirror = j < i;
    const int a = mirror ? j : i, c = mirror ? i : j;
    const int g = (c - nold) / SC_NC, cc = (c - nold) % SC_NC;
    double2 v = make_double2(0.0, 0.0);
    for (int b = 0; b < nband; ++b) {
        const double2 pv = part[((((long)s * ngroups + g) * nband + b) * NTP + a) * SC_NC + cc];
        v.x += pv.x;
        v.y += pv.y;
    }
    if (i == j) v.y = 0.0;
    if (mirror) v.y = -v.y;
    if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(&ws.flags[s], 2);
    rnew[base + (long)i * NTP + j] = v;
}

// R_new as the inputs of the tissue basis (FP32 copy) and of the assembly (the
// deflated Gram with zero tissue blocks), row i per work-group.
template <int NTP>
__global__ void __launch_bounds__(256) k_cov_export(Workspace ws, const double2* rnew) {
    constexpr int NTE = NTP + REXT;
    const int s = blockIdx.x, i = blockIdx.y;
    const long base = (long)s * NTP * NTP;
    for (int j = threadIdx.x; j < NTE; j += 256) {
        double2 v = make_double2(0.0, 0.0);
        if (i < NTP && j < NTP) {
            v = rnew[base + (long)i * NTP + j];
            ws.rwin[base + (long)i * NTP + j] = make_float2((float)v.x, (float)v.y);
        }
        ws.rext[(long)s * NTE * NTE + (long)i * NTE + j] = v;
    }
}

template <int NTP>
static void stream_dispatch(const Workspace& ws, const double2* rold, double2* rnew, double2* part, int hop,
                            hipStream_t st) {
    const int ngroups = (hop + SC_NC - 1) / SC_NC;
    const int nband = ngroups == 1 ? (NTP / SC_NC > 4 ? NTP / SC_NC : 4) : 1;
    if (hop <= 8)
        hipLaunchKernelGGL((k_cov_new<NTP, 8>), dim3(ws.S, ngroups, nband), dim3(256), 0, st, ws, part, hop,
                           ngroups, nband);
    else
        hipLaunchKernelGGL((k_cov_new<NTP, SC_NC>), dim3(ws.S, ngroups, nband), dim3(256), 0, st, ws, part, hop,
                           ngroups, nband);
    hipLaunchKernelGGL((k_cov_finish<NTP>), dim3(ws.S, NTP), dim3(256), 0, st, ws, (const double2*)rold, rnew,
                       (const double2*)part, hop, ngroups, nband);
    hipLaunchKernelGGL((k_cov_export<NTP>), dim3(ws.S, NTP + REXT), dim3(256), 0, st, ws, (const double2*)rnew);
}

size_t stream_partial_elems(int S, int ntp) {
    // ngroups * nband <= max(4, ntp / 16): ngroups <= ntp / 16 with one band,
    // or one group in max(4, ntp / 16) bands
    const size_t gb = ntp / SC_NC > 4 ? (size_t)(ntp / SC_NC) : 4;
    return (size_t)S * gb * ntp * SC_NC;
}

hipError_t launch_cov_stream(const Workspace& ws, const double2* rold, double2* rnew, double2* part, int hop,
                             hipStream_t st) {
    switch (ws.ntp) {
        case 32: stream_dispatch<32>(ws, rold, rnew, part, hop, st); break;
        case 64: stream_dispatch<64>(ws, rold, rnew, part, hop, st); break;
        case 96: stream_dispatch<96>(ws, rold, rnew, part, hop, st); break;
        case 128: stream_dispatch<128>(ws, rold, rnew, part, hop, st); break;
        case 160: stream_dispatch<160>(ws, rold, rnew, part, hop, st); break;
        case 208: stream_dispatch<208>(ws, rold, rnew, part, hop, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lcf
