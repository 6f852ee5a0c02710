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

constexpr int SC_PB = 64;    // pixels per LDS batch
constexpr int SC_NC = 16;    // new columns per work-group

// Work-group (s, g, b): new columns j0 .. j0 + 15 (j0 = nt - h + 16 g) of
// subset s over row band b of its box. Thread i accumulates
// sum_x w_x^2 conj(s(x, t_i)) s(x, t_j) for its row i and every column of the
// group; the band's sums go to part[s][g][b][i][16].
template <int NTP>
__global__ void __launch_bounds__(256) k_cov_new(Workspace ws, double2* part, int hop, int ngroups, int nband) {
    __shared__ float2 sr[NTP * (SC_PB + 1)];
    __shared__ double w2[SC_PB];
    const int s = blockIdx.x, g = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
    const SubsetDesc sd = ws.sub[s];
    const int nt = sd.nt;
    const int j0 = nt - hop + SC_NC * g;
    const int ncol = min(SC_NC, nt - j0);
    const int nrow = sd.y1 - sd.y0 + 1;
    const int r0 = (int)((long)nrow * b / nband), r1 = (int)((long)nrow * (b + 1) / nband);
    const int q0 = r0 * sd.bw, q1 = r1 * sd.bw;
    const double* wy = ws.wtab + sd.wy_off;
    const double* wx = ws.wtab + sd.wx_off;
    const long npix = (long)sd.ny * sd.nx;
    double2 acc[SC_NC];
#pragma unroll
    for (int c = 0; c < SC_NC; ++c) acc[c] = make_double2(0.0, 0.0);
    for (int qb = q0; qb < q1; qb += SC_PB) {
        __syncthreads();   // previous batch consumed
        for (int e = tid; e < nt * SC_PB; e += 256) {
            const int t = e / SC_PB, p = e % SC_PB, q = qb + p;
            float2 v = make_float2(0.f, 0.f);
            if (q < q1) {
                const int y = sd.y0 + q / sd.bw, x = sd.x0 + q % sd.bw;
                v = sd.iq[(long)t * npix + (long)y * sd.nx + x];
            }
            sr[t * (SC_PB + 1) + p] = v;
        }
        if (tid < SC_PB) {
            const int q = qb + tid;
            double w = 0.0;
            if (q < q1) {
                const int y = sd.y0 + q / sd.bw, x = sd.x0 + q % sd.bw;
                w = sd.flat ? 1.0 : wy[y - sd.y0] * wx[x - sd.x0];
            }
            w2[tid] = w * w;
        }
        __syncthreads();
        if (tid < nt) {
            for (int p = 0; p < SC_PB; ++p) {
                const float2 a = sr[tid * (SC_PB + 1) + p];
                const double ww = w2[p];
                const double ar = (double)a.x * ww, ai = -(double)a.y * ww;   // w^2 conj(a)
#pragma unroll
                for (int c = 0; c < SC_NC; ++c) {
                    if (c < ncol) {
                        const float2 bv = sr[(j0 + c) * (SC_PB + 1) + p];
                        const double br = (double)bv.x, bi = (double)bv.y;
                        acc[c].x = fma(ar, br, fma(-ai, bi, acc[c].x));
                        acc[c].y = fma(ar, bi, fma(ai, br, acc[c].y));
                    }
                }
            }
        }
    }
    if (tid < NTP) {
        double2* o = part + ((((long)s * ngroups + g) * nband + b) * NTP + tid) * SC_NC;
#pragma unroll
        for (int c = 0; c < SC_NC; ++c) o[c] = tid < nt ? acc[c] : make_double2(0.0, 0.0);
    }
}

// Column j of R_new for subset s (thread = row): a retained column copies the
// retained rows from R_old shifted by h; a new column adds the band partials in
// band order for rows i <= j and writes R[i][j] and R[j][i] = conj (the
// diagonal real), so each entry is written by exactly one work-group.
template <int NTP>
__global__ void __launch_bounds__(256) k_cov_finish(Workspace ws, const double2* rold, double2* rnew,
                                                    const double2* part, int hop, int ngroups, int nband) {
    const int s = blockIdx.x, j = blockIdx.y, i = threadIdx.x;
    const int nt = ws.sub[s].nt;
    if (j >= nt || i >= nt) return;
    const long base = (long)s * NTP * NTP;
    const int nold = nt - hop;
    if (j < nold) {
        if (i < nold) rnew[base + (long)i * NTP + j] = rold[base + (long)(i + hop) * NTP + (j + hop)];
        return;
    }
    if (i > j) return;
    const int g = (j - nold) / SC_NC, c = (j - nold) % SC_NC;
    double2 v = make_double2(0.0, 0.0);
    for (int b = 0; b < nband; ++b) {
        const double2 pv = part[((((long)s * ngroups + g) * nband + b) * NTP + i) * SC_NC + c];
        v.x += pv.x;
        v.y += pv.y;
    }
    if (i == j) v.y = 0.0;
    if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(&ws.flags[s], 2);
    rnew[base + (long)i * NTP + j] = v;
    rnew[base + (long)j * NTP + i] = make_double2(v.x, -v.y);
}

// R_new as the inputs of the tissue basis (FP32 copy) and of the assembly (the
// deflated Gram with zero tissue blocks), column j per work-group.
template <int NTP>
__global__ void __launch_bounds__(256) k_cov_export(Workspace ws, const double2* rnew) {
    constexpr int NTE = NTP + REXT;
    const int s = blockIdx.x, j = blockIdx.y;
    const long base = (long)s * NTP * NTP;
    for (int i = threadIdx.x; i < NTE; i += 256) {
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
    const int nband = ngroups == 1 ? 4 : 1;
    hipLaunchKernelGGL((k_cov_new<NTP>), dim3(ws.S, ngroups, nband), dim3(256), 0, st, ws, part, hop, ngroups,
                       nband);
    hipLaunchKernelGGL((k_cov_finish<NTP>), dim3(ws.S, NTP), dim3(256), 0, st, ws, (const double2*)rold, rnew,
                       (const double2*)part, hop, ngroups, nband);
    hipLaunchKernelGGL((k_cov_export<NTP>), dim3(ws.S, NTP + REXT), dim3(256), 0, st, ws, (const double2*)rnew);
}

size_t stream_partial_elems(int S, int ntp) {
    // ngroups * nband <= max(4, ntp / 16) groups of 16 columns
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
