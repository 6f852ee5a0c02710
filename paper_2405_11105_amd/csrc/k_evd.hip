// FP64 small-matrix stages of each subset: window tables (Eq. 11), the tissue
// basis used to deflate the covariance, the deflated-basis assembly of R, and
// the batched Hermitian eigen-decomposition (Eq. 2) by one-sided Jacobi.
#include <type_traits>

#include "lcf_internal.h"
#include "lcf_kernels.h"

namespace lcf {

// ------------------------------------------------------------------ windows
// 1-D factors of the separable Gaussian window of Eq. 11 over the subset box.
__global__ void __launch_bounds__(256) k_windows(Workspace ws) {
    const SubsetDesc sd = ws.sub[blockIdx.x];
    const int ny = sd.y1 - sd.y0 + 1, nx = sd.x1 - sd.x0 + 1;
    if (threadIdx.x == 0) ws.flags[blockIdx.x] = 0;
    for (int i = threadIdx.x; i < ny; i += blockDim.x) {
        const double d = (double)(sd.y0 + i) - sd.cy;
        ws.wtab[sd.wy_off + i] = sd.flat ? 1.0 : exp(-(d * d) / (2.0 * sd.sy * sd.sy));
    }
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double d = (double)(sd.x0 + i) - sd.cx;
        ws.wtab[sd.wx_off + i] = sd.flat ? 1.0 : exp(-(d * d) / (2.0 * sd.sx * sd.sx));
    }
}

// ------------------------------------------------------------------ tissue basis
// Approximate dominant eigenvectors of the pass-1 covariance by subspace
// iteration + Rayleigh-Ritz, keep the r of them whose Ritz value exceeds
// rho * theta_1, and build an exactly unitary basis Q = H_0 ... H_{r-1} whose
// first r columns span them (complex Householder reflectors, FP64). Any V_r is
// valid for the deflation identity C_w = C' + (C_w V_r) V_r^H; accuracy of V_r
// only decides how small C' is.

// Tiny Hermitian EVD (order RMAX = 8, zero-padded) by parallel cyclic Jacobi on
// one wave: lane l holds H[l / 8][l % 8] and Z[l / 8][l % 8]. A sweep is 7
// rounds of 4 disjoint pairs (circle schedule). All rotations of a round are
// formed from the entries before it (disjoint pairs do not touch each other's
// 2 x 2 blocks), then H <- H J, Z <- Z J and H <- J^H H for every pair, with
//   J = [[c, s], [-s conj(e), c conj(e)]] for pair p < q,  e = H_pq / |H_pq|,
//   theta = (H_qq - H_pp) / (2 |H_pq|), t = sign(theta) / (|theta| + sqrt(theta^2 + 1)),
//   c = 1 / sqrt(t^2 + 1), s = t c.
static_assert(RMAX == 8, "one wave holds the 8 x 8 Ritz matrix");

__device__ __forceinline__ int circle_partner(int m, int k) {
    // players 1..7 sit at positions (m - 1 + k) mod 7 and player 0 at the hub;
    // the hub meets position 0, position i meets position 7 - i
    if (m == 0) return ((7 - k) % 7) + 1;
    const int pos = (m - 1 + k) % 7;
    if (pos == 0) return 0;
    return ((7 - pos - k + 14) % 7) + 1;
}

__device__ __forceinline__ double2 shfl2(double2 v, int src) {
    return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__device__ __forceinline__ void jac8_params(double2 h, int p, int q, double2& j00, double2& j01, double2& j10,
                                            double2& j11) {
    const double2 apq = shfl2(h, p * 8 + q);
    const double hpp = __shfl(h.x, p * 9, 64), hqq = __shfl(h.x, q * 9, 64);
    const double mag = sqrt(cabs2(apq));
    j00 = make_double2(1.0, 0.0);
    j01 = make_double2(0.0, 0.0);
    j10 = make_double2(0.0, 0.0);
    j11 = make_double2(1.0, 0.0);
    if (mag > 0.0) {
        const double2 ph = make_double2(apq.x / mag, apq.y / mag);
        const double theta = (hqq - hpp) / (2.0 * mag);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        j00 = make_double2(c, 0.0);
        j01 = make_double2(sn, 0.0);
        j10 = make_double2(-sn * ph.x, sn * ph.y);
        j11 = make_double2(c * ph.x, -c * ph.y);
    }
}

__device__ void wave_heev8(double2& h, double2& z, int lane) {
    const int i = lane >> 3, j = lane & 7;
    z = make_double2(i == j ? 1.0 : 0.0, 0.0);
    for (int sweep = 0; sweep < 40; ++sweep) {
        const double a = cabs2(h);
        const double tot = wave_sum_x(a), off = wave_sum_x(i != j ? a : 0.0);
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int k = 0; k < 7; ++k) {
            const int pj = circle_partner(j, k), pi = circle_partner(i, k);
            const int pc = j < pj ? j : pj, qc = j < pj ? pj : j;
            const int pr = i < pi ? i : pi, qr = i < pi ? pi : i;
            double2 c00, c01, c10, c11, r00, r01, r10, r11;
            jac8_params(h, pc, qc, c00, c01, c10, c11);
            jac8_params(h, pr, qr, r00, r01, r10, r11);
            // columns: H J, Z J
            const double2 hp = shfl2(h, i * 8 + pc), hq = shfl2(h, i * 8 + qc);
            const double2 zp = shfl2(z, i * 8 + pc), zq = shfl2(z, i * 8 + qc);
            if (j == pc) {
                h = cadd(cmul(hp, c00), cmul(hq, c10));
                z = cadd(cmul(zp, c00), cmul(zq, c10));
            } else {
                h = cadd(cmul(hp, c01), cmul(hq, c11));
                z = cadd(cmul(zp, c01), cmul(zq, c11));
            }
            // rows: J^H (H J)
            const double2 gp = shfl2(h, pr * 8 + j), gq = shfl2(h, qr * 8 + j);
            h = i == pr ? cadd(cmulc(r00, gp), cmulc(r10, gq)) : cadd(cmulc(r01, gp), cmulc(r11, gq));
        }
    }
}

template <int NTP>
__global__ void __launch_bounds__(256, NTP <= 128 ? 4 : NTP <= 160 ? 3 : 2) k_tissue(Workspace ws, double rho, int iters) {
    constexpr int XR = (NTP + 63) / 64;         // rows per lane in the one-wave passes
    __shared__ double2 X[NTP * RMAX];
    __shared__ double2 Y[NTP * RMAX];
    __shared__ double2 H[RMAX * RMAX], Z[RMAX * RMAX];
    __shared__ double th[RMAX], tsh[RMAX];
    __shared__ double dg[NTP];
    __shared__ int piv[RMAX], order[RMAX];
    __shared__ double red[32];
    __shared__ int sh_r;
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const SubsetDesc sd = ws.sub[s];
    const int nt = sd.nt;
    const float2* Rf = ws.rwin + (long)s * NTP * NTP;
    auto R = [&](long i) { const float2 f = Rf[i]; return make_double2((double)f.x, (double)f.y); };
    double2* hv = ws.hv + (long)s * RMAX * NTP;
    double* htau = ws.htau + (long)s * RMAX;
    const int ns = nt < RMAX ? nt : RMAX;

    // start block: the columns of R at its ns largest diagonal entries, found by
    // the rank of each entry (ties by index; NaN ranks last)
    for (int t = tid; t < nt; t += 256) {
        const double d = R((long)t * NTP + t).x;
        dg[t] = d == d ? d : -1e300;
    }
    if (tid < RMAX) piv[tid] = tid;
    __syncthreads();
    for (int t = tid; t < nt; t += 256) {
        const double d = dg[t];
        int rk = 0;
        for (int u = 0; u < nt; ++u) rk += (dg[u] > d) || (dg[u] == d && u < t);
        if (rk < ns) piv[rk] = t;
    }
    __syncthreads();
    for (int e = tid; e < NTP * RMAX; e += 256) {
        const int t = e / RMAX, j = e % RMAX;
        // R[t][piv] = conj(R[piv][t])
        X[e] = (t < nt && j < ns) ? cconj(R((long)piv[j] * NTP + t)) : make_double2(0.0, 0.0);
    }
    __syncthreads();

    // modified Gram-Schmidt, two passes, in the registers of wave 0
    auto orthonormalize = [&]() {
        if (wave == 0) {
            double2 x[XR][RMAX];
#pragma unroll
            for (int i = 0; i < XR; ++i)
#pragma unroll
                for (int j = 0; j < RMAX; ++j) {
                    const int t = lane + 64 * i;
                    x[i][j] = t < nt ? X[t * RMAX + j] : make_double2(0.0, 0.0);
                }
            for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
                for (int j = 0; j < RMAX; ++j) {
                    if (j >= ns) continue;
#pragma unroll
                    for (int q = 0; q < j; ++q) {
                        double dr = 0.0, di = 0.0;                 // conj(x_q) x_j
#pragma unroll
                        for (int i = 0; i < XR; ++i) {
                            dr = fma(x[i][q].x, x[i][j].x, fma(x[i][q].y, x[i][j].y, dr));
                            di = fma(x[i][q].x, x[i][j].y, fma(-x[i][q].y, x[i][j].x, di));
                        }
                        const double2 dot = make_double2(wave_sum_x(dr), wave_sum_x(di));
#pragma unroll
                        for (int i = 0; i < XR; ++i) x[i][j] = cfma(x[i][q], make_double2(-dot.x, -dot.y), x[i][j]);
                    }
                    double n2 = 0.0;
#pragma unroll
                    for (int i = 0; i < XR; ++i) n2 += cabs2(x[i][j]);
                    const double nrm = sqrt(wave_sum_x(n2));
                    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll
                    for (int i = 0; i < XR; ++i) x[i][j] = cscale(x[i][j], inv);
                }
            }
#pragma unroll
            for (int i = 0; i < XR; ++i)
#pragma unroll
                for (int j = 0; j < RMAX; ++j) {
                    const int t = lane + 64 * i;
                    if (t < NTP) X[t * RMAX + j] = x[i][j];
                }
        }
        __syncthreads();
    };
    // Y = R X, coalesced through R[u][t] = conj(R[t][u]); two threads per row t
    // (alternate u), combined by a lane swap
    auto apply_R = [&]() {
        for (int t0 = 0; t0 < nt; t0 += 128) {
            const int t = t0 + (tid >> 1), half = tid & 1;
            double2 acc[RMAX];
#pragma unroll
            for (int j = 0; j < RMAX; ++j) acc[j] = make_double2(0.0, 0.0);
            if (t < nt) {
                // eight entries of R requested together, the next eight (raw FP32)
                // in flight while these are used (beyond nt: zero, times a finite
                // row of X)
                auto fetchR = [&](int u0, float2 (&f)[8]) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int u = u0 + 2 * q;
                        f[q] = u < nt ? Rf[(long)u * NTP + t] : make_float2(0.f, 0.f);
                    }
                };
                float2 rf[8];
                fetchR(half, rf);
                for (int u0 = half; u0 < nt; u0 += 16) {
                    float2 rc[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) rc[q] = rf[q];
                    if (u0 + 16 < nt) fetchR(u0 + 16, rf);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int u = u0 + 2 * q < nt ? u0 + 2 * q : 0;
                        const double2 rv = make_double2((double)rc[q].x, -(double)rc[q].y);
#pragma unroll
                        for (int j = 0; j < RMAX; ++j) acc[j] = cfma(rv, X[u * RMAX + j], acc[j]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < RMAX; ++j) {
                acc[j].x += dpp_d<0xB1>(acc[j].x);
                acc[j].y += dpp_d<0xB1>(acc[j].y);
            }
            if (t < nt && half == 0) {
#pragma unroll
                for (int j = 0; j < RMAX; ++j) Y[t * RMAX + j] = acc[j];
            }
        }
        __syncthreads();
    };

    for (int it = 0; it < iters; ++it) {
        orthonormalize();
        apply_R();
        for (int e = tid; e < nt * RMAX; e += 256) X[e] = Y[e];
        __syncthreads();
    }
    orthonormalize();
    apply_R();
    if (tid < RMAX * RMAX) {
        const int i = tid / RMAX, j = tid % RMAX;
        double2 acc = make_double2(0.0, 0.0);
        if (i < ns && j < ns)
            for (int t = 0; t < nt; ++t) acc = cfmac(X[t * RMAX + i], Y[t * RMAX + j], acc);
        H[tid] = acc;
    }
    __syncthreads();
    if (wave == 0) {
        // Hermitian part (rounding), then the Ritz pairs
        const int i = lane >> 3, j = lane & 7;
        const double2 a = H[lane], b = H[j * RMAX + i];
        double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        if (i == j) h.y = 0.0;
        double2 z;
        wave_heev8(h, z, lane);
        Z[lane] = z;
        if (i == j) th[i] = h.x;
    }
    __syncthreads();
    if (tid == 0) {
        // order descending, then the rank cut
        for (int i = 0; i < ns; ++i) order[i] = i;
        for (int i = 0; i < ns; ++i)
            for (int j = i + 1; j < ns; ++j)
                if (th[order[j]] > th[order[i]]) { const int tmp = order[i]; order[i] = order[j]; order[j] = tmp; }
        int r = 0;
        const double t1 = ns > 0 ? th[order[0]] : 0.0;
        if (rho > 0.0 && t1 > 0.0 && isfinite(t1))
            while (r < ns && th[order[r]] > rho * t1) ++r;
        sh_r = r;
    }
    __syncthreads();
    const int r = sh_r;
    // U = X Z (ordered), kept in Y
    for (int e = tid; e < nt * RMAX; e += 256) {
        const int t = e / RMAX, j = e % RMAX;
        double2 acc = make_double2(0.0, 0.0);
        if (j < r)
            for (int i = 0; i < ns; ++i) acc = cfma(X[t * RMAX + i], Z[i * RMAX + order[j]], acc);
        Y[e] = acc;
    }
    __syncthreads();
    // Householder QR of U[:, :r], thread t holding row t (each thread updates
    // only its own rows; the barriers of the block sums order the rest)
    static_assert(NTP <= 256, "one row per thread");
    const int t = tid;
    const bool trow = t < nt;
    for (int j = 0; j < r; ++j) {
        const double2 yj = (trow && t >= j) ? Y[t * RMAX + j] : make_double2(0.0, 0.0);
        const double nx2 = block_sum_x(cabs2(yj), red);
        const double nrm = sqrt(nx2);
        const double2 x0 = Y[j * RMAX + j];
        const double ax0 = sqrt(cabs2(x0));
        const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
        const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
        // v = x - alpha e_j ; v^H v = 2 (|x|^2 + |x| |x0|)
        const double vv = 2.0 * (nx2 + nrm * ax0);
        const double tau = vv > 0.0 ? 2.0 / vv : 0.0;
        const double2 v = t == j ? csub(x0, alpha) : (t > j && trow ? yj : make_double2(0.0, 0.0));
        if (t < NTP) hv[(long)j * NTP + t] = v;
        if (tid == 0) {
            htau[j] = tau;
            tsh[j] = tau;
        }
        // apply H_j to columns j+1..r-1 of U
        for (int c = j + 1; c < r; ++c) {
            const double2 yc = (trow && t >= j) ? Y[t * RMAX + c] : make_double2(0.0, 0.0);
            const double2 dot = block_sum2_x(cfmac(v, yc, make_double2(0.0, 0.0)), red);
            if (trow && t >= j) Y[t * RMAX + c] = cfma(v, make_double2(-tau * dot.x, -tau * dot.y), yc);
        }
    }
    // explicit V_r = H_0 ... H_{r-1} [e_0 .. e_{r-1}]
    for (int e = tid; e < NTP * RMAX; e += 256) {
        const int te = e / RMAX, j = e % RMAX;
        X[e] = make_double2((te == j && j < r) ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int j = r - 1; j >= 0; --j) {
        const double tau = tsh[j];
        const double2 vj = trow ? hv[(long)j * NTP + t] : make_double2(0.0, 0.0);   // this thread's own write
        for (int c = 0; c < r; ++c) {
            const double2 xc = (trow && t >= j) ? X[t * RMAX + c] : make_double2(0.0, 0.0);
            const double2 dot = block_sum2_x(cfmac(vj, xc, make_double2(0.0, 0.0)), red);
            if (trow && t >= j) X[t * RMAX + c] = cfma(vj, make_double2(-tau * dot.x, -tau * dot.y), xc);
        }
    }
    __syncthreads();
    for (int e = tid; e < NTP * RMAX; e += 256) {
        ws.vr64[(long)s * NTP * RMAX + e] = X[e];
        ws.vr32[(long)s * NTP * RMAX + e] = make_float2((float)X[e].x, (float)X[e].y);
    }
    if (tid == 0) ws.rank[s] = r;
}

// ------------------------------------------------------------------ assembly
// R = R2 + G' V_r^H + V_r G'^H + V_r (Y^H Y) V_r^H   (exact for C_w = C' + Y V_r^H)
// written as R2 + E V_r^H + V_r E^H with E = G' + V_r (Y^H Y) / 2, then
// B = Q^H R Q = H_{r-1} .. H_0 R H_0 .. H_{r-1} (Hermitian rank-2 updates).
// keep_r: also write R (original basis) to the P area, for the covariance
// diagnostics exported right after this stage (the EVD reuses that area).
// Up to 128 frames B is held in registers, 4 rows x 8 columns of it per thread
// over 512 threads (8 x 8 per thread over 256 needed AGPRs as spill space and
// left one wave per SIMD); beyond, 256 threads work on it in global memory.
template <int NTP>
struct AsmCfg {
    static constexpr int NTHR = NTP <= 128 ? 512 : 256;
    static constexpr int RA = 2048 / NTHR;      // rows per thread (register path)
};

template <int NTP>
__global__ void __launch_bounds__(AsmCfg<NTP>::NTHR) k_assemble(Workspace ws, int keep_r) {
    constexpr int NTE = NTP + REXT;
    constexpr int NTHR = AsmCfg<NTP>::NTHR, RA = AsmCfg<NTP>::RA, NRG = NTHR / 16;
    __shared__ double2 E[NTP * RMAX];
    __shared__ double2 V[NTP * RMAX];
    __shared__ double2 P[2][NTP];
    __shared__ double2 vh[RMAX * NTP];
    __shared__ double red[2][NRG > 16 ? NRG : 16];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nt = ws.sub[s].nt;
    const int r = ws.rank[s];
    const double2* X = ws.rext + (long)s * NTE * NTE;
    double2* B = ws.bmat + (long)s * NTP * NTP;
    for (int e = tid; e < NTP * RMAX; e += NTHR) {
        V[e] = ws.vr64[(long)s * NTP * RMAX + e];
        const int j = e / NTP;
        vh[e] = j < r ? ws.hv[(long)s * RMAX * NTP + e] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < NTP * RMAX; e += NTHR) {
        const int t = e / RMAX, j = e % RMAX;
        double2 acc = make_double2(0.0, 0.0);
        if (t < nt && j < r) {
            acc = X[(long)t * NTE + NTP + j];
            for (int i = 0; i < r; ++i)
                acc = cadd(acc, cscale(cmul(V[t * RMAX + i], X[(long)(NTP + i) * NTE + NTP + j]), 0.5));
        }
        E[e] = acc;
    }
    __syncthreads();
    if constexpr (NTP <= 128) {
        // R, then B, in registers: thread (ti, ui) holds rows RA ti + a, columns
        // ui + 16 b. Per reflector: p = B v by lane shuffles over the 16 lanes of
        // a row group, v^H p and the rows of p through LDS (one barrier), then
        // B -= tau (v w^H + w v^H), w = p - (tau / 2)(v^H p) v.
        const int ti = threadIdx.x >> 4, ui = threadIdx.x & 15;
        double2 acc[RA][8];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int t = RA * ti + a, u = ui + 16 * b;
                double2 v = make_double2(0.0, 0.0);
                if (t < nt && u < nt) {
                    v = X[(long)t * NTE + u];
                    for (int j = 0; j < r; ++j) {
                        v = cadd(v, cmulc(V[u * RMAX + j], E[t * RMAX + j]));   // E_tj conj(V_uj)
                        v = cadd(v, cmulc(E[u * RMAX + j], V[t * RMAX + j]));   // V_tj conj(E_uj)
                    }
                    if (t == u) v.y = 0.0;
                }
                if (keep_r && t < NTP && u < NTP) ws.pmat[(long)s * NTP * NTP + (long)t * NTP + u] = v;
                acc[a][b] = v;
            }
        for (int j = 0; j < r; ++j) {
            const double tau = ws.htau[(long)s * RMAX + j];
            const double2* v = vh + j * NTP;
            // column-outer loops keep one column's v (and w) live at a time
            double2 pa[RA];
#pragma unroll
            for (int a = 0; a < RA; ++a) pa[a] = make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int u = ui + 16 * b;
                const double2 vu = u < NTP ? v[u] : make_double2(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < RA; ++a) pa[a] = cadd(pa[a], cmul(acc[a][b], vu));
            }
            double kpart = 0.0;
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                // sum over the 16 lanes of the row (lane moves within it)
                pa[a].x += dpp_d<0xB1>(pa[a].x);
                pa[a].y += dpp_d<0xB1>(pa[a].y);
                pa[a].x += dpp_d<0x4E>(pa[a].x);
                pa[a].y += dpp_d<0x4E>(pa[a].y);
                pa[a].x += dpp_d<0x141>(pa[a].x);
                pa[a].y += dpp_d<0x141>(pa[a].y);
                pa[a].x += dpp_d<0x140>(pa[a].x);
                pa[a].y += dpp_d<0x140>(pa[a].y);
                const int t = RA * ti + a;
                if (ui == 0 && t < NTP) P[j & 1][t] = pa[a];
                if (t < NTP) kpart += cmulc(v[t], pa[a]).x;
            }
            if (ui == 0) red[j & 1][ti] = kpart;
            __syncthreads();
            double K = 0.0;
#pragma unroll
            for (int q = 0; q < NRG; ++q) K += red[j & 1][q];
            const double hk = 0.5 * tau * K;
            double2 vt[RA], wt[RA];
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const int t = RA * ti + a;
                vt[a] = t < NTP ? v[t] : make_double2(0.0, 0.0);
                wt[a] = t < NTP ? csub(P[j & 1][t], cscale(vt[a], hk)) : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int u = ui + 16 * b;
                const double2 vu = u < NTP ? v[u] : make_double2(0.0, 0.0);
                const double2 wu = u < NTP ? csub(P[j & 1][u], cscale(vu, hk)) : make_double2(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < RA; ++a) {
                    // B -= tau (v_t conj(w_u) + w_t conj(v_u))
                    const double2 d = cadd(cmulc(wu, vt[a]), cmulc(vu, wt[a]));
                    double2 x = csub(acc[a][b], cscale(d, tau));
                    if (RA * ti + a == u) x.y = 0.0;
                    acc[a][b] = x;
                }
            }
        }
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int t = RA * ti + a, u = ui + 16 * b;
                if (t < NTP && u < NTP) B[(long)t * NTP + u] = (t < nt && u < nt) ? acc[a][b] : make_double2(0.0, 0.0);
            }
    } else {
        for (int e = tid; e < NTP * NTP; e += 256) {
            const int t = e / NTP, u = e % NTP;
            double2 b = make_double2(0.0, 0.0);
            if (t < nt && u < nt) {
                b = X[(long)t * NTE + u];
                for (int j = 0; j < r; ++j) {
                    b = cadd(b, cmulc(V[u * RMAX + j], E[t * RMAX + j]));   // E_tj conj(V_uj)
                    b = cadd(b, cmulc(E[u * RMAX + j], V[t * RMAX + j]));   // V_tj conj(E_uj)
                }
                if (t == u) b.y = 0.0;
            }
            B[e] = b;
            if (keep_r) ws.pmat[(long)s * NTP * NTP + e] = b;
        }
        __syncthreads();
        for (int j = 0; j < r; ++j) {
            const double tau = ws.htau[(long)s * RMAX + j];
            for (int t = tid; t < NTP; t += 256) vh[t] = ws.hv[((long)s * RMAX + j) * NTP + t];
            __syncthreads();
            // p = B v, via B[t][u] = conj(B[u][t])
            for (int t = tid; t < nt; t += 256) {
                double2 acc = make_double2(0.0, 0.0);
                for (int u = 0; u < nt; ++u) acc = cadd(acc, cmulc(B[(long)u * NTP + t], vh[u]));
                P[0][t] = acc;
            }
            __syncthreads();
            double part = 0.0;
            for (int t = tid; t < nt; t += 256) part += cmulc(vh[t], P[0][t]).x;
            const double K = block_sum(part, &red[0][0]);
            for (int t = tid; t < nt; t += 256) P[0][t] = csub(P[0][t], cscale(vh[t], 0.5 * tau * K));
            __syncthreads();
            for (int e = tid; e < nt * NTP; e += 256) {
                const int t = e / NTP, u = e % NTP;
                if (u >= nt) continue;
                // B -= tau (v_t conj(w_u) + w_t conj(v_u))
                const double2 d = cadd(cmulc(P[0][u], vh[t]), cmulc(vh[u], P[0][t]));
                double2 b = csub(B[e], cscale(d, tau));
                if (t == u) b.y = 0.0;
                B[e] = b;
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ Jacobi
// One-sided (Hestenes) Jacobi on G = B: rotate column pairs until all columns
// are mutually orthogonal; then G = W Lambda with W unitary, so lambda_j =
// ||g_j|| and w_j = g_j / lambda_j (B is positive semi-definite). Columns are
// stored contiguously (column-major, read as conj of the row-major Hermitian
// input). Pairs follow the round-robin tournament order, nt/2 disjoint pairs
// per step, one wave per pair, lanes over rows. Because the B of a subset is
// taken in the tissue-deflated basis, large and small eigenvalues sit in nearly
// decoupled blocks and the small columns keep their accuracy.
__device__ __forceinline__ void rr_pair(int step, int k, int n, int& p, int& q) {
    const int m = n - 1;
    int a, b;
    if (k == 0) { a = 0; b = 1 + step % m; }
    else { a = 1 + (step + k) % m; b = 1 + (step - k + m) % m; }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

constexpr int JAC_THREADS = 1024;
constexpr int JAC_LDS_NT = 100;   // nt*nt*16 bytes must fit the 160 KiB LDS

// Stopping rule: a sweep without rotations (every pair passes the relative
// test |g_p^H g_q| <= nt*u*||g_p|| ||g_q||), or stagnation at the rounding floor:
// when R is ill-conditioned and not graded, the small columns carry absolute
// rounding noise of order u*||R|| and the relative test cannot be met; after four
// sweeps, a sweep whose largest relative off-diagonal is below 1e-6 and has not
// dropped fourfold ends the iteration. Only the sweep cap raises the flag.
template <bool IN_LDS>
__device__ void jacobi_core(double2* G, int nt, int ld, int max_sweeps, int* sweeps_out, int* flag_out) {
    __shared__ int rot;
    __shared__ double wmax[32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int n = nt + (nt & 1);
    const double tol = (double)nt * 1.1102230246251565e-16;
    int sweep = 0;
    bool converged = false;
    double prev_off = 1e300;
    for (; sweep < max_sweeps; ++sweep) {
        if (threadIdx.x == 0) rot = 0;
        double my_off = 0.0;
        __syncthreads();
        for (int step = 0; step < n - 1; ++step) {
            for (int k = wave; k < n / 2; k += nw) {
                int p, q;
                rr_pair(step, k, n, p, q);
                if (q >= nt) continue;
                double2* gp = G + (long)p * ld;
                double2* gq = G + (long)q * ld;
                double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
                for (int row = lane; row < nt; row += 64) {
                    const double2 a = gp[row], b = gq[row];
                    al += cabs2(a);
                    be += cabs2(b);
                    gr += a.x * b.x + a.y * b.y;
                    gi += a.x * b.y - a.y * b.x;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                gr = wave_sum(gr);
                gi = wave_sum(gi);
                const double mag = sqrt(gr * gr + gi * gi);
                const double scale = sqrt(al * be);
                if (scale > 0.0) my_off = fmax(my_off, mag / scale);
                if (!(mag > tol * scale)) continue;
                const double zeta = (be - al) / (2.0 * mag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                const double er = gr / mag, ei = -gi / mag;     // e^{-i phi}
                for (int row = lane; row < nt; row += 64) {
                    const double2 a = gp[row], b = gq[row];
                    const double2 bt = make_double2(b.x * er - b.y * ei, b.x * ei + b.y * er);
                    gp[row] = make_double2(c * a.x - sn * bt.x, c * a.y - sn * bt.y);
                    gq[row] = make_double2(sn * a.x + c * bt.x, sn * a.y + c * bt.y);
                }
                if (lane == 0) atomicAdd(&rot, 1);
            }
            __syncthreads();
        }
        if (lane == 0) wmax[wave] = my_off;
        __syncthreads();
        double off = 0.0;
        for (int i = 0; i < nw; ++i) off = fmax(off, wmax[i]);
        const bool stagnant = sweep >= 3 && off < 1e-6 && off > 0.25 * prev_off;
        prev_off = off;
        if (rot == 0 || stagnant) { converged = true; ++sweep; break; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *sweeps_out = sweep;
        if (!converged) atomicOr(flag_out, 4);
    }
    __syncthreads();
}

__device__ void jacobi_finish(const double2* G, int nt, int ld, double* lam_out, double2* vout, int ldv,
                              bool col_major);

// ------------------------------------------------------------------ register-resident Jacobi
// The same one-sided Jacobi with the matrix held in VGPRs: NW waves hold 16
// columns each (two half-blocks of 8: "top" slots 0-7 and "bottom" slots 8-15),
// lane l holds rows l + 64 i (i < RPL). A sweep is (1) all pairs inside each
// half-block (7 steps of the circle method on 8 slots) and (2) 2 NW - 1 rounds in
// which every wave pairs each top column with each bottom column (8 steps,
// bottom slots rotated by one after each step), after which half-blocks move
// between waves through LDS following the circle method over the 2 NW
// half-blocks (half-block 0 stays in place). Each step handles 8 disjoint pairs:
// lane partial sums, a transposed butterfly that leaves dot product (l >> 1) in
// lane l, rotation parameters in lanes 0-7, broadcast by readlane.
// The lane-swap instructions on a double: returns the two swapped operands.
template <int M>
__device__ __forceinline__ void swap_d(double a, double b, double& x, double& y) {
    const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
    const unsigned alo = (unsigned)(ab & 0xffffffff), ahi = (unsigned)(ab >> 32);
    const unsigned blo = (unsigned)(bb & 0xffffffff), bhi = (unsigned)(bb >> 32);
    unsigned x0, x1, y0, y1;
    if constexpr (M == 32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        x0 = lo[0]; y0 = lo[1]; x1 = hi[0]; y1 = hi[1];
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        x0 = lo[0]; y0 = lo[1]; x1 = hi[0]; y1 = hi[1];
    }
    x = __longlong_as_double((long long)(((unsigned long long)x1 << 32) | x0));
    y = __longlong_as_double((long long)(((unsigned long long)y1 << 32) | y0));
}

// 1/sqrt(x) and 1/x to double precision: the hardware estimates refined by two
// Newton steps each (y <- y + y (1 - x y^2) / 2 and y <- y + y (1 - x y)).
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double r = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, r, y);
    }
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

template <int RPL>
struct JCols {
    double2 x[16][RPL];
};

// Pair slots of a step. MODE 0 (inside half-blocks): (0,7) (1,6) (2,5) (3,4) and
// the same in the bottom half; MODE 1 (across): (i, 8 + i).
__host__ __device__ constexpr int pslot_a(int mode, int k) { return mode == 0 ? (k < 4 ? k : 4 + k) : k; }
__host__ __device__ constexpr int pslot_b(int mode, int k) { return mode == 0 ? (k < 4 ? 7 - k : 19 - k) : 8 + k; }

// Rotate 4 disjoint pairs (k = G..G+3) of the wave's registers. The 16 lane
// partial sums are ordered quantity-major (4 q + k: q = |a|^2, |b|^2, Re a^H b,
// Im a^H b) so that after the transposed reduction lane l holds quantity l >> 4
// of pair (l >> 2) & 3, and two lane swaps bring all four quantities of pair k
// to lanes 4k..4k+3 of the first row.
template <int RPL, int MODE, int G>
__device__ __forceinline__ void jac_step4(JCols<RPL>& c, int lane, double tol, int& nrot, double& offmax) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const double2 a = c.x[pslot_a(MODE, G + k)][i], b = c.x[pslot_b(MODE, G + k)][i];
            al = fma(a.x, a.x, fma(a.y, a.y, al));
            be = fma(b.x, b.x, fma(b.y, b.y, be));
            gr = fma(a.x, b.x, fma(a.y, b.y, gr));
            gi = fma(a.x, b.y, fma(-a.y, b.x, gi));
        }
        v[0 + k] = al;
        v[4 + k] = be;
        v[8 + k] = gr;
        v[12 + k] = gi;
    }
    // transposed reduction: lane bit 5 <- index bit 3 (lane swap 32), bit 4 <- bit 2
    // (lane swap 16), bit 3 <- bit 1 (row mirror), bit 2 <- bit 0 (half-row
    // mirror), then a plain sum over the quad. Selects work on named scalars so
    // that none turns into an indexed register access.
    double w8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) w8[j] = swap_sum<32>(v[j], v[j + 8]);
    double u[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = swap_sum<16>(w8[j], w8[j + 4]);
    const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
    const double u0 = u[0], u1 = u[1], u2 = u[2], u3 = u[3];
    const double z0 = (h8 ? u2 : u0) + dpp_d<0x140>(h8 ? u0 : u2);
    const double z1 = (h8 ? u3 : u1) + dpp_d<0x140>(h8 ? u1 : u3);
    double tot = (h4 ? z1 : z0) + dpp_d<0x141>(h4 ? z0 : z1);
    tot += dpp_d<0x4E>(tot);
    tot += dpp_d<0xB1>(tot);
    // rows of tot: |a|^2, |b|^2, Re, Im; bring rows 1-3 to row 0
    double r0, r1, s0, s1, t0, t1;
    swap_d<32>(tot, tot, r0, r1);      // r0 rows: al be al be; r1: gr gi gr gi
    swap_d<16>(r0, r1, s0, s1);        // s1 rows: be gi be gi
    swap_d<16>(r1, r1, t0, t1);        // t1 rows: gi gi gi gi (row 0 = gi)
    const double al = tot, be = s1, gr = r1, gi = t1;
    // rotation of pair (lane >> 2) & 3 from squared quantities (no square roots or
    // divisions beyond three reciprocal square roots and one reciprocal)
    const double m2 = fma(gr, gr, gi * gi), ab = al * be;
    const bool rot = m2 > tol * tol * ab;
    const double im = rsq_nr(m2);
    const double zeta = 0.5 * (be - al) * im;
    const double z2 = fma(zeta, zeta, 1.0);
    const double t = (zeta >= 0 ? 1.0 : -1.0) * rcp_nr(fabs(zeta) + z2 * rsq_nr(z2));
    const double cr = rsq_nr(fma(t, t, 1.0));
    const double cc = rot ? cr : 1.0, ss = rot ? cr * t : 0.0;
    const double er = rot ? gr * im : 1.0, ei = rot ? -gi * im : 0.0;
    const double off2 = ab > 0.0 ? m2 / ab : 0.0;
    const unsigned long long rb = __ballot(rot && lane < 16 && (lane & 3) == 0);
    nrot += __popcll(rb);
    if (lane < 16) offmax = fmax(offmax, off2);      // lane-local; reduced once per sweep
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double C = rdl(cc, 4 * q), S = rdl(ss, 4 * q), ER = rdl(er, 4 * q), EI = rdl(ei, 4 * q);
        const double SR = S * ER, SI = S * EI, CR = C * ER, CI = C * EI;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const double2 a = c.x[pslot_a(MODE, G + q)][i], b = c.x[pslot_b(MODE, G + q)][i];
            c.x[pslot_a(MODE, G + q)][i] =
                make_double2(fma(C, a.x, -fma(SR, b.x, -SI * b.y)), fma(C, a.y, -fma(SR, b.y, SI * b.x)));
            c.x[pslot_b(MODE, G + q)][i] =
                make_double2(fma(S, a.x, fma(CR, b.x, -CI * b.y)), fma(S, a.y, fma(CR, b.y, CI * b.x)));
        }
    }
}

template <int RPL, int MODE>
__device__ __forceinline__ void jac_step8(JCols<RPL>& c, int lane, double tol, int& nrot, double& offmax) {
    jac_step4<RPL, MODE, 0>(c, lane, tol, nrot, offmax);
    jac_step4<RPL, MODE, 4>(c, lane, tol, nrot, offmax);
}

template <int RPL, int NW>
__global__ void __launch_bounds__(64 * NW) k_jacobi_reg(Workspace ws, int max_sweeps, int only_flag) {
    if (only_flag != 0 && (ws.flags[blockIdx.x] & only_flag) == 0) return;   // not selected: whole block exits
    constexpr int ROWS = 64 * RPL;
    constexpr int SLOT = 8 * ROWS;                     // double2 per half-block
    __shared__ double2 xch[(NW + 1) * SLOT];
    __shared__ int idx[NW + 1];
    __shared__ int s_rot[NW];
    __shared__ double s_off[NW];
    const int s = blockIdx.x, lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar branches
    const int nt = ws.sub[s].nt, ntp = ws.ntp;
    const double2* B = ws.bmat + (long)s * ntp * ntp;
    double2* Gout = ws.wvec + (long)s * ntp * ntp;
    const double tol = (double)nt * 1.1102230246251565e-16;

    int my_top = 2 * wave, my_bot = 2 * wave + 1;
    JCols<RPL> c;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int col = (j < 8 ? my_top : my_bot) * 8 + (j & 7);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            c.x[j][i] = (row < nt && col < nt) ? cconj(B[(long)col * ntp + row]) : make_double2(0.0, 0.0);
        }
    }
    int sweep = 0;
    bool converged = false;
    double prev_off = 1e300;
    for (; sweep < max_sweeps; ++sweep) {
        int nrot = 0;
        double offmax = 0.0;
        // (1) pairs inside each half-block: circle method, slot 0 (and 8) fixed
#pragma unroll 1
        for (int st = 0; st < 7; ++st) {
            jac_step8<RPL, 0>(c, lane, tol, nrot, offmax);
#pragma unroll
            for (int h = 0; h < 16; h += 8) {
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const double2 t7 = c.x[h + 7][i];
#pragma unroll
                    for (int j = 7; j > 1; --j) c.x[h + j][i] = c.x[h + j - 1][i];
                    c.x[h + 1][i] = t7;
                }
            }
        }
        // (2) cross rounds
#pragma unroll 1
        for (int rd = 0; rd < 2 * NW - 1; ++rd) {
#pragma unroll 1
            for (int st = 0; st < 8; ++st) {
                jac_step8<RPL, 1>(c, lane, tol, nrot, offmax);
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const double2 t0 = c.x[8][i];
#pragma unroll
                    for (int j = 8; j < 15; ++j) c.x[j][i] = c.x[j + 1][i];
                    c.x[15][i] = t0;
                }
            }
            if (rd == 2 * NW - 2) break;      // the last round needs no move
            // move half-blocks (circle method, half-block at wave 0 top fixed)
            auto put = [&](int slot, int base) {
#pragma unroll
                for (int j = 0; j < 8; ++j)
#pragma unroll
                    for (int i = 0; i < RPL; ++i) xch[slot * SLOT + j * ROWS + lane + 64 * i] = c.x[base + j][i];
            };
            auto get = [&](int slot, int base) {
#pragma unroll
                for (int j = 0; j < 8; ++j)
#pragma unroll
                    for (int i = 0; i < RPL; ++i) c.x[base + j][i] = xch[slot * SLOT + j * ROWS + lane + 64 * i];
            };
            __syncthreads();
            // phase 1: tops move right; wave 0's bottom becomes wave 1's top
            if (wave >= 1) { put(wave, 0); if (lane == 0) idx[wave] = my_top; }
            else { put(0, 8); if (lane == 0) idx[0] = my_bot; }
            __syncthreads();
            if (wave >= 1) { get(wave - 1, 0); my_top = idx[wave - 1]; }
            __syncthreads();
            // phase 2: bottoms move left; the last wave's old top becomes its bottom
            if (wave == NW - 1) {
                put(NW, 8);
                if (lane == 0) idx[NW] = my_bot;
                get(NW - 1, 8);                 // old top written in phase 1
                my_bot = idx[NW - 1];
            } else if (wave >= 1) {
                put(wave, 8);
                if (lane == 0) idx[wave] = my_bot;
            }
            __syncthreads();
            if (wave <= NW - 2) {
                const int src = (wave == NW - 2) ? NW : wave + 1;
                get(src, 8);
                my_bot = idx[src];
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) offmax = fmax(offmax, __shfl_xor(offmax, m, 64));
        if (lane == 0) { s_rot[wave] = nrot; s_off[wave] = sqrt(offmax); }
        __syncthreads();
        int tr = 0;
        double off = 0.0;
        for (int w = 0; w < NW; ++w) { tr += s_rot[w]; off = fmax(off, s_off[w]); }
        const bool stagnant = sweep >= 3 && off < 1e-6 && off > 0.25 * prev_off;
        prev_off = off;
        __syncthreads();
        if (tr == 0 || stagnant) { converged = true; ++sweep; break; }
    }
    // write columns back (column-major, stride ntp)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int col = (j < 8 ? my_top : my_bot) * 8 + (j & 7);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            if (row < nt && col < nt) Gout[(long)col * ntp + row] = c.x[j][i];
        }
    }
    if (threadIdx.x == 0) {
        ws.sweeps[s] = sweep;
        if (!converged) atomicOr(&ws.flags[s], 4);
    }
    __syncthreads();
    jacobi_finish(Gout, nt, ntp, ws.lam + (long)s * ntp, ws.bmat + (long)s * ntp * ntp, ntp, true);
}


// ------------------------------------------------------------------ tridiagonal EVD
// Subset EVD (Eq. 2) through a real symmetric tridiagonal matrix:
//  1. Householder reduction B = Q T Q^H, Q = H_0 .. H_{n-3}, H_j = I - tau v v^H,
//     with the two-sided update A <- A - v q^H - q v^H (p = tau A v,
//     q = p - (tau / 2)(v^H p) v); the vectors go to scratch.
//  2. T = D T_r D^H with a diagonal unitary D makes the off-diagonal real >= 0.
//     (Steps 1 and 2: k_heev_tri_reduce up to 128 frames, the matrix in VGPRs,
//     columns dealt to the waves cyclically (slot k of wave w holds column
//     NW k + w, lane l rows l + 64 i); k_heev_big_reduce below, the matrix in
//     global memory.)
//  3. Eigenvalues of T_r by multisection of Sturm counts (4 lanes per
//     eigenvalue, 5 sub-intervals per round), sorted descending by construction
//     (k_heev_sturm, for both).
//  4. Each eigenvector of T_r from a twisted factorisation
//     (T_r - lambda I) = N_r Delta_r N_r^T at the twist index r of smallest
//     |gamma_r|, one lane per eigenvalue (one O(n) solve, no iteration).
//  5. Eigenvectors of B: y = Q D z, the reflectors applied in reverse order.
//     (Steps 4 and 5: k_heev_tri_vecs, after the weights.)
// Only the components whose weight differs from 1 enter the projector, so only
// their vectors are formed (step 4 and 5, after the weights). A subset where one
// of them has a neighbour closer than 1e-12 lambda_1 (where such vectors would
// lose orthogonality) keeps its B and is flagged for the Jacobi kernel, which
// then runs on it alone; near-equal eigenvalues among the others (the noise
// floor's smallest spacings) need no vectors and no fallback.
// The scratch of a subset (the second half of its projector slot) holds the
// tridiagonal form: d, |e|, |e|^2, Re D, Im D (N each), then pivmin and the
// Gershgorin interval.
constexpr int FLAG_EVD_FALLBACK = 16;

template <int RPL, int NW>
__global__ void __launch_bounds__(64 * NW) k_heev_tri_reduce(Workspace ws) {
    constexpr int N = 16 * NW;             // padded size held (columns)
    static_assert(64 * RPL >= N, "rows per lane cover the padded size");
    __shared__ double2 psh[2][NW][N];      // per-wave partials of A v, by the parity of the step
    __shared__ double2 colb[2][N];         // the column the next reflector comes from, by parity
    __shared__ double2 vqw[NW][2][16];     // each wave's copy of v and q at its own columns
    __shared__ double red[2];
    __shared__ double dsh[N], esh[N], e2sh[N];
    __shared__ double2 phs[N];             // complex e_j, then D
    __shared__ double bnd[2];
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nt = ws.sub[s].nt;
    double2* Bm = ws.bmat + (long)s * N * N;
    double2* H = ws.wvec + (long)s * N * N;                 // Householder vectors, tau in element 0
    double* trid = reinterpret_cast<double*>(ws.pmat + (long)s * N * N) + N * N;   // tridiagonal form

    // slot k: column NW k + wave, so that every wave keeps columns to update
    // until the last steps
    double2 A[16][RPL];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int col = NW * k + wave;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            A[k][i] = (row < nt && col < nt) ? cconj(Bm[(long)col * N + row]) : make_double2(0.0, 0.0);
        }
    }

    // ---- 1. Householder reduction, one barrier per column: every wave forms
    // the next reflector itself from the column its owner published a step
    // earlier (updating it by the current step first), so no wave waits for
    // another one's reflector.
    // The reflector of column jj (rows jj + 1 ..) from x, that column of the
    // current matrix at this lane's rows; the same bits in every wave.
    // (straight-line code, so that it can interleave with the update; `record`
    // stores what it found)
    auto form = [&](int jj, const double2 (&x)[RPL], double2 (&v)[RPL], double& xjj, double2& ej)
                    __attribute__((always_inline)) -> double {
        double s2 = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            if (row > jj + 1 && row < nt) s2 += cabs2(x[i]);
        }
        s2 = wave_sum_x(s2);
        double2 t1 = x[0];
        double t0 = x[0].x;
#pragma unroll
        for (int i = 1; i < RPL; ++i) {
            if (i == ((jj + 1) >> 6)) t1 = x[i];
            if (i == (jj >> 6)) t0 = x[i].x;
        }
        const double2 x0 = make_double2(rdl(t1.x, (jj + 1) & 63), rdl(t1.y, (jj + 1) & 63));
        xjj = rdl(t0, jj & 63);
        // (a subnormal |x0|^2 or alpha (alpha + |x0|) counts as zero: the
        // hardware reciprocal estimates take normal numbers)
        constexpr double tiny = 2.2250738585072014e-308;
        const double n0 = cabs2(x0);
        const double r0 = n0 >= tiny ? rsq_nr(n0) : 0.0;
        const double ax0 = n0 * r0;
        const double alpha = sqrt(s2 + n0);
        const double2 ph = n0 >= tiny ? cscale(x0, r0) : make_double2(1.0, 0.0);
        const double den = alpha * (alpha + ax0);
        const double tau = den >= tiny ? rcp_nr(den) : 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            v[i] = row <= jj ? make_double2(0.0, 0.0) : (row == jj + 1 ? cadd(x0, cscale(ph, alpha)) : x[i]);
        }
        ej = cscale(ph, -alpha);                                    // complex e_jj for now
        return tau;
    };
    // reflector jj to scratch (one wave), d_jj and e_jj to LDS
    auto record = [&](int jj, const double2 (&v)[RPL], double tau, double xjj, double2 ej)
                      __attribute__((always_inline)) {
        if (wave == jj % NW) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int row = lane + 64 * i;
                if (row < N) H[(long)jj * N + row] = row == 0 ? make_double2(tau, 0.0) : v[i];   // row 0 of v_j is zero: holds tau
            }
            if (lane == 0) {
                dsh[jj] = xjj;
                phs[jj] = ej;
            }
        }
    };
    // this lane's values of a vector at the wave's own columns into vqw[wave][h]
    auto own_cols = [&](const double2 (&u)[RPL], int h) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            if (row < N && row % NW == wave) vqw[wave][h][row / NW] = u[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // (A is only ever indexed by compile-time constants, outside any lambda, so
    // that it stays in registers)

    double2 vr[RPL];                        // v_j at this lane's rows
    double tau = 0.0;
    if (nt > 2) {
        // columns 0 and 1: slot 0 of waves 0 and 1
        if (wave < 2) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int row = lane + 64 * i;
                if (row < N) colb[wave ^ 1][row] = A[0][i];
            }
        }
        __syncthreads();
        double2 x[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            x[i] = row < N ? colb[1][row] : make_double2(0.0, 0.0);
        }
        double xjj;
        double2 ej;
        tau = form(0, x, vr, xjj, ej);
        record(0, vr, tau, xjj, ej);
    }
    // Two passes over the steps: in the second (j >= 63, two row blocks) the
    // first row block holds only finished rows, where v and q vanish, so it is
    // left as it is (rows i < ILO).
    int j = 0;
#pragma unroll
    for (int ILO = 0; ILO < RPL; ++ILO) {
        const int jend = ILO + 1 < RPL ? 63 : 1 << 30;
        for (; j + 2 < nt && j < jend; ++j) {
            const int par = j & 1;
            // slots k >= kf hold the columns > j (v vanishes at columns <= j,
            // which are finished: a group of 4 slots with one of them active is
            // updated whole, which changes only finished columns that no step
            // reads again)
            const int kf = j < wave ? 0 : (j - wave) / NW + 1;
            own_cols(vr, 0);
            // partial A v over this wave's columns (slots in groups of 4 from the
            // group of slot kf: v is zero at the finished columns among them)
            double2 acc[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) acc[i] = make_double2(0.0, 0.0);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (4 * g + 3 >= kf) {
                    double2 vc[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) vc[u] = vqw[wave][0][4 * g + u];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int i = ILO; i < RPL; ++i) {
                            const double2 a = A[4 * g + u][i];
                            acc[i].x = fma(a.x, vc[u].x, fma(-a.y, vc[u].y, acc[i].x));
                            acc[i].y = fma(a.x, vc[u].y, fma(a.y, vc[u].x, acc[i].y));
                        }
                }
            }
            // (rows <= j are finished: p and q there reach only other finished
            // rows, so neither is formed)
#pragma unroll
            for (int i = ILO; i < RPL; ++i) {
                const int row = lane + 64 * i;
                if (row > j && row < N) psh[par][wave][row] = acc[i];
            }
            __syncthreads();
            // p = tau A v for this lane's rows, q = p - (tau / 2) (v^H p) v
            double2 qr[RPL];
            double kr = 0.0, ki = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int row = lane + 64 * i;
                double2 p = make_double2(0.0, 0.0);
                if (i >= ILO && row > j && row < N) {
                    double2 pw[NW];
#pragma unroll
                    for (int w = 0; w < NW; ++w) pw[w] = psh[par][w][row];
#pragma unroll
                    for (int w = 0; w < NW; ++w) p = cadd(p, pw[w]);
                }
                qr[i] = cscale(p, tau);
                kr = fma(vr[i].x, qr[i].x, fma(vr[i].y, qr[i].y, kr));       // conj(v) p
                ki = fma(vr[i].x, qr[i].y, fma(-vr[i].y, qr[i].x, ki));
            }
            {
                // both sums at once: lanes below 32 end with the sum of kr, the others with ki's
                double t = swap_sum<32>(kr, ki);
                t += dpp_d<0xB1>(t);
                t += dpp_d<0x4E>(t);
                t += dpp_d<0x141>(t);
                t += dpp_d<0x140>(t);
                t = swap_sum<16>(t, t);
                kr = rdl(t, 0);
                ki = rdl(t, 32);
            }
            const double2 K = make_double2(0.5 * tau * kr, 0.5 * tau * ki);
#pragma unroll
            for (int i = 0; i < RPL; ++i) qr[i] = csub(qr[i], cmul(K, vr[i]));
            own_cols(qr, 1);
            // the next reflector, from column j + 1 after this step's update
            double2 vn[RPL];
            double taun = 0.0, xn = 0.0;
            double2 en = make_double2(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < RPL; ++i) vn[i] = make_double2(0.0, 0.0);
            if (j + 3 < nt) {
                const int r = j + 1;
                double2 qs = qr[0], vs = vr[0];
#pragma unroll
                for (int i = 1; i < RPL; ++i)
                    if (i == (r >> 6)) { qs = qr[i]; vs = vr[i]; }
                const double2 qc = make_double2(rdl(qs.x, r & 63), rdl(qs.y, r & 63));
                const double2 vc = make_double2(rdl(vs.x, r & 63), rdl(vs.y, r & 63));
                double2 x[RPL];
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const int row = lane + 64 * i;
                    const double2 a = row < N ? colb[par][row] : make_double2(0.0, 0.0);
                    double ax = a.x, ay = a.y;
                    ax = fma(-vr[i].x, qc.x, fma(-vr[i].y, qc.y, ax));
                    ay = fma(-vr[i].y, qc.x, fma(vr[i].x, qc.y, ay));
                    ax = fma(-qr[i].x, vc.x, fma(-qr[i].y, vc.y, ax));
                    ay = fma(-qr[i].y, vc.x, fma(qr[i].x, vc.y, ay));
                    x[i] = make_double2(ax, ay);
                }
                taun = form(r, x, vn, xn, en);
            }
            // A -= v q^H + q v^H on this wave's columns
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (4 * g + 3 >= kf) {
                    double2 vc[4], qc[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        vc[u] = vqw[wave][0][4 * g + u];
                        qc[u] = vqw[wave][1][4 * g + u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int i = ILO; i < RPL; ++i) {
                            const int k = 4 * g + u;
                            double ax = A[k][i].x, ay = A[k][i].y;
                            ax = fma(-vr[i].x, qc[u].x, fma(-vr[i].y, qc[u].y, ax));
                            ay = fma(-vr[i].y, qc[u].x, fma(vr[i].x, qc[u].y, ay));
                            ax = fma(-qr[i].x, vc[u].x, fma(-qr[i].y, vc[u].y, ax));
                            ay = fma(-qr[i].y, vc[u].x, fma(qr[i].x, vc[u].y, ay));
                            A[k][i] = make_double2(ax, ay);
                        }
                }
            }
            if (j + 3 < nt) record(j + 1, vn, taun, xn, en);
            // column j + 2 as this step leaves it, for the reflector after next
            // (held by wave (j + 2) % NW in slot (j + 2) / NW)
            if (j + 4 < nt && wave == (j + 2) % NW) {
                const int ks = (j + 2) / NW;
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    if (k == ks) {
#pragma unroll
                        for (int i = 0; i < RPL; ++i) {
                            const int row = lane + 64 * i;
                            if (row < N) colb[par ^ 1][row] = A[k][i];
                        }
                    }
            }
#pragma unroll
            for (int i = 0; i < RPL; ++i) vr[i] = vn[i];
            tau = taun;
        }
    }
    // last 2 x 2 block: d_{nt-2}, d_{nt-1}, e_{nt-2}
    {
        const int r0 = nt - 2, r1 = nt - 1;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int col = NW * k + wave;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int row = lane + 64 * i;
                if (row == r0 && col == r0) dsh[r0] = A[k][i].x;
                if (row == r1 && col == r1) dsh[r1] = A[k][i].x;
                if (row == r1 && col == r0) phs[r0] = A[k][i];
            }
        }
    }
    __syncthreads();
    // ---- 2. real tridiagonal (wave 0, element j in lane j % 64, register j / 64):
    // |e_j|, the phases D (d_0 = 1, d_{j+1} = d_j e_j / |e_j|, a prefix product
    // by a shuffle scan) and the Gershgorin interval
    if (wave == 0) {
        double2 u[RPL];
        double ae[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int j = lane + 64 * i;
            const double2 e = j + 1 < nt ? phs[j] : make_double2(0.0, 0.0);
            ae[i] = sqrt(cabs2(e));
            u[i] = ae[i] > 0.0 ? cscale(e, 1.0 / ae[i]) : make_double2(1.0, 0.0);
            if (j + 1 < nt) {
                esh[j] = ae[i];
                e2sh[j] = ae[i] * ae[i];
            }
        }
        // inclusive products within each 64-element segment, then across segments
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const double2 t = make_double2(__shfl_up(u[i].x, off, 64), __shfl_up(u[i].y, off, 64));
                if (lane >= off) u[i] = cmul(t, u[i]);
            }
        double2 carry = make_double2(1.0, 0.0);
        double2 dexc[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const double2 incl = cmul(carry, u[i]);
            const double2 prev = make_double2(__shfl_up(incl.x, 1, 64), __shfl_up(incl.y, 1, 64));
            // per component: a select between two double2 values becomes a select of
            // their addresses and puts both on the stack
            dexc[i] = make_double2(lane == 0 ? carry.x : prev.x, lane == 0 ? carry.y : prev.y);
            carry = make_double2(rdl(incl.x, 63), rdl(incl.y, 63));
        }
        double lo = 1e300, hi = -1e300, emax = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int j = lane + 64 * i;
            if (j < N) phs[j] = dexc[i];
            if (j < nt) {
                const double aprev = __shfl_up(ae[i], 1, 64);
                const double aprv = lane == 0 ? (i > 0 ? rdl(ae[i - 1 >= 0 ? i - 1 : 0], 63) : 0.0) : aprev;
                const double rad = (j > 0 ? aprv : 0.0) + (j + 1 < nt ? ae[i] : 0.0);
                lo = fmin(lo, dsh[j] - rad);
                hi = fmax(hi, dsh[j] + rad);
                if (j + 1 < nt) emax = fmax(emax, ae[i] * ae[i]);
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, m, 64));
            hi = fmax(hi, __shfl_xor(hi, m, 64));
            emax = fmax(emax, __shfl_xor(emax, m, 64));
        }
        if (lane == 0) {
            const double margin = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
            bnd[0] = lo - margin;
            bnd[1] = hi + margin;
            red[0] = 1e-290 * fmax(1.0, emax);                         // pivmin
        }
    }
    __syncthreads();
    // the tridiagonal form (d, |e|, |e|^2, D), pivmin and the Gershgorin interval
    for (int i = tid; i < N; i += 64 * NW) {
        trid[i] = dsh[i];
        trid[N + i] = esh[i];
        trid[2 * N + i] = e2sh[i];
        trid[3 * N + i] = phs[i].x;
        trid[4 * N + i] = phs[i].y;
    }
    if (tid == 0) {
        trid[5 * N] = red[0];
        trid[5 * N + 1] = bnd[0];
        trid[5 * N + 2] = bnd[1];
    }
}

// Step 3 for both reduction kernels. NTHR Sturm counts at grid points (the
// lower Gershgorin bound, then geometric steps from hi 2^-64 up to hi) bracket
// every eigenvalue; then multisection, lanes 4k .. 4k+3 for the k-th largest,
// 4 points and 5 sub-intervals per round, until the bracket is no wider than
// (hi - lo) 1.7e-17 (24 rounds from the Gershgorin interval reach it, below
// the rounding of the largest eigenvalue). Four lanes per eigenvalue in every
// batch, so that a packet's eigenvalues do not depend on what it is batched
// with: two lanes and three sub-intervals per round need about 66 counts per
// eigenvalue instead of 90 (1.73 -> 1.70 ms for the four-packet step at 128
// frames) but about 33 dependent rounds instead of 22, which one packet's 256
// subsets cannot hide (0.18 -> 0.25 ms). Each count is a dependent chain of
// nt divisions: the kernel holds few registers, so several work-groups per CU
// hide that latency (inside the reduction kernels two waves per SIMD did).
template <int N, int NTHR>
__global__ void __launch_bounds__(NTHR) k_heev_sturm(Workspace ws) {
    static_assert(NTHR >= 4 * N, "four lanes per eigenvalue");
    __shared__ double dsh[N], e2sh[N];
    __shared__ int gcnt[NTHR];                 // Sturm counts at the bracketing grid
    __shared__ int offdiag;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nt = ws.sub[s].nt;
    const double* trid = reinterpret_cast<const double*>(ws.pmat + (long)s * N * N) + N * N;
    if (tid == 0) offdiag = 0;
    __syncthreads();
    for (int i = tid; i < N; i += NTHR) {
        dsh[i] = trid[i];
        e2sh[i] = trid[2 * N + i];
        if (i + 1 < nt && e2sh[i] != 0.0) offdiag = 1;
    }
    if (tid == 0) ws.sweeps[s] = 0;
    __syncthreads();
    if (!offdiag) {
        // T is diagonal (an all-zero packet, for one): its eigenvalues are the
        // diagonal exactly, in descending order (ties by index)
        if (tid < nt) {
            const double v = dsh[tid];
            int rank = 0;
            for (int j = 0; j < nt; ++j) rank += dsh[j] > v || (dsh[j] == v && j < tid);
            ws.lam[(long)s * N + rank] = v;
        }
        return;
    }
    const double pivmin = trid[5 * N], lo = trid[5 * N + 1], hi = trid[5 * N + 2];
    auto sturm = [&](double x) {
        double q = dsh[0] - x;
        int c = q < 0.0;
        for (int i = 1; i < nt; ++i) {
            if (fabs(q) < pivmin) q = -pivmin;
            q = (dsh[i] - x) - e2sh[i - 1] * rcp_nr(q);
            c += q < 0.0;
        }
        return c;
    };
    auto grid = [&](int g) {
        if (hi <= 0.0) return lo + (hi - lo) * (double)g / (double)(NTHR - 1);
        if (g == 0) return lo;
        return fmax(lo, hi * exp2(-64.0 * (double)(NTHR - 1 - g) / (double)(NTHR - 2)));
    };
    gcnt[tid] = sturm(grid(tid));
    __syncthreads();
    const int k = tid >> 2, m = tid & 3;
    const int target = nt - 1 - k;                                 // index among ascending
    // counts are nondecreasing along the grid: the last point with count <= target
    int g0 = 0, g1 = NTHR - 1;                                     // gcnt[g0] <= target < gcnt[g1]
    while (g1 - g0 > 1) {
        const int gm = (g0 + g1) >> 1;
        if (gcnt[gm] <= target) g0 = gm;
        else g1 = gm;
    }
    double a = grid(g0), b = g1 == NTHR - 1 ? hi : grid(g1);
    const double tol = (hi - lo) * 1.7e-17;
    for (int it = 0; it < 24 && b - a > tol; ++it) {
        const double h = (b - a) * 0.2;
        const double x = a + (double)(m + 1) * h;
        const int cnt = k < nt ? sturm(x) : 0;
        // the points left of the eigenvalue are those with count <= target
        int le = cnt <= target;
        le += __builtin_amdgcn_mov_dpp(le, 0xB1, 0xF, 0xF, false);          // lane ^ 1
        le += __builtin_amdgcn_mov_dpp(le, 0x4E, 0xF, 0xF, false);          // lane ^ 2
        const double na = a + (double)le * h;
        b = le == 4 ? b : a + (double)(le + 1) * h;
        a = na;
    }
    if (m == 0 && k < nt) ws.lam[(long)s * N + k] = 0.5 * (a + b);
}

// Eigenvectors of the subsets solved by the tridiagonal path (steps 4 and 5), for
// the components whose weight differs from 1 (all of them when `all` is set):
// only those enter the projector P = I - W' diag(1 - w) W'^H.
template <int RPL, int NW>
__global__ void __launch_bounds__(64 * (NW < 4 ? NW : 4)) k_heev_tri_vecs(Workspace ws, int all) {
    constexpr int N = 16 * NW;
    constexpr int NWV = NW < 4 ? NW : 4;   // waves: groups of SG selected columns at a time
    constexpr int SG = 16 * NWV;
    static_assert(64 * NWV >= N, "one thread per component for the selection");
    static_assert(64 * RPL >= N, "rows per lane cover the padded size");
    __shared__ double dsh[N], esh[N], e2sh[N];
    __shared__ double2 phs[N];
    __shared__ double lamsh[N], insh[SG];
    __shared__ double dml[N * SG];         // [i][slot in group]: D- of the slot's eigenvalue, then its z
    __shared__ int act[N];
    __shared__ int wcnt[NWV];
    __shared__ int cluster;
    __shared__ double2 wsh[NWV][16];       // per wave: v^H y of its 16 columns
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) cluster = 0;
    const int nt = ws.sub[s].nt;
    double2* Bm = ws.bmat + (long)s * N * N;
    const double2* H = ws.wvec + (long)s * N * N;
    double* Dp = reinterpret_cast<double*>(ws.pmat + (long)s * N * N);   // [i][slot]: D+
    const double* trid = Dp + N * N;
    const double* wts = ws.wts + (long)s * N;
    for (int i = tid; i < N; i += 64 * NWV) {
        dsh[i] = trid[i];
        esh[i] = trid[N + i];
        e2sh[i] = trid[2 * N + i];
        phs[i] = make_double2(trid[3 * N + i], trid[4 * N + i]);
        lamsh[i] = ws.lam[(long)s * N + i];
    }
    const double pivmin = trid[5 * N];
    // selected components in ascending order, by ballots
    const bool flag = tid < nt && (all || fabs(1.0 - wts[tid < N ? tid : 0]) > 1e-17);
    const unsigned long long mask = __ballot(flag);
    if (lane == 0) wcnt[wave] = __popcll(mask);
    __syncthreads();
    int nact = 0, off = 0;
    for (int w = 0; w < NWV; ++w) {
        off += w < wave ? wcnt[w] : 0;
        nact += wcnt[w];
    }
    if (flag) {
        act[off + __popcll(mask & ((1ull << lane) - 1ull))] = tid;
        // a selected component with a neighbour closer than 1e-12 lambda_1
        const double tol = 1e-12 * fabs(lamsh[0]);
        if ((tid > 0 && lamsh[tid - 1] - lamsh[tid] <= tol) || (tid + 1 < nt && lamsh[tid] - lamsh[tid + 1] <= tol))
            cluster = 1;
    }
    __syncthreads();
    if (cluster) {                                  // B stays for the Jacobi kernel
        if (tid == 0) atomicOr(&ws.flags[s], FLAG_EVD_FALLBACK);
        return;
    }
    for (int g0 = 0; g0 < nact; g0 += SG) {
    const int cnt = nact - g0 < SG ? nact - g0 : SG;
    // ---- 4. eigenvectors of T_r by twisted factorisation (lane k); D- and then
    // z live in LDS, D+ goes to scratch and is read back eight at a time
    if (tid < cnt) {
        const int k = tid;                         // slot in the group; the eigenvalue is act[g0 + k]
        const double lam = lamsh[act[g0 + k]];
        double q = dsh[nt - 1] - lam;
        dml[(nt - 1) * SG + k] = q;
        for (int i = nt - 2; i >= 0; --i) {
            if (fabs(q) < pivmin) q = -pivmin;
            q = (dsh[i] - lam) - e2sh[i] * rcp_nr(q);
            dml[i * SG + k] = q;
        }
        double p = dsh[0] - lam;
        Dp[k] = p;
        int r = 0;
        double g = fabs(dml[k]);
        for (int i = 0; i + 1 < nt; ++i) {
            if (fabs(p) < pivmin) p = -pivmin;
            p = (dsh[i + 1] - lam) - e2sh[i] * rcp_nr(p);
            Dp[(long)(i + 1) * N + k] = p;
            const double gam = p + dml[(i + 1) * SG + k] - (dsh[i + 1] - lam);
            if (fabs(gam) < g) { g = fabs(gam); r = i + 1; }
        }
        // z_r = 1; below r from D+, above r from D- (each D- is read before its
        // slot takes the z value)
        double z = 1.0, nrm = 1.0;
        dml[r * SG + k] = 1.0;
        for (int i = r - 1; i >= 0; i -= 8) {
            double dv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) dv[u] = i - u >= 0 ? Dp[(long)(i - u) * N + k] : 1.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (i - u >= 0) {
                    double d = dv[u];
                    if (fabs(d) < pivmin) d = -pivmin;
                    z = -esh[i - u] * rcp_nr(d) * z;
                    dml[(i - u) * SG + k] = z;
                    nrm += z * z;
                }
            }
        }
        z = 1.0;
        for (int i = r; i + 1 < nt; ++i) {
            double d = dml[(i + 1) * SG + k];
            if (fabs(d) < pivmin) d = -pivmin;
            z = -esh[i] * rcp_nr(d) * z;
            dml[(i + 1) * SG + k] = z;
            nrm += z * z;
        }
        insh[k] = rsq_nr(nrm);
    }
    __syncthreads();
    // ---- 5. y = Q D z in registers, reflectors in reverse order (the next
    // reflector is loaded while the current one is applied)
    double2 A[16][RPL];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int col = 16 * wave + c;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            A[c][i] = (row < nt && col < cnt) ? cscale(phs[row], dml[row * SG + col] * insh[col])
                                              : make_double2(0.0, 0.0);
        }
    }
    double2 vn[RPL];
    double taun = 0.0;
    auto hload = [&](int j) {
        taun = H[(long)j * N].x;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int row = lane + 64 * i;
            vn[i] = (row > j && row < N) ? H[(long)j * N + row] : make_double2(0.0, 0.0);
        }
    };
    if (16 * wave < cnt) {                        // the wave holds selected columns
    if (nt >= 3) hload(nt - 3);
    for (int j = nt - 3; j >= 0; --j) {
        const double tauj = taun;
        double2 vr[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) vr[i] = vn[i];
        if (j > 0) hload(j - 1);
        // w_c = v^H y_c for this wave's 16 columns: lane partials, then a
        // transposed reduction leaving value (l >> 1) in lane l
        double v32[32];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            double ar = 0.0, ai = 0.0;                                 // conj(v) y
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                ar = fma(vr[i].x, A[c][i].x, fma(vr[i].y, A[c][i].y, ar));
                ai = fma(vr[i].x, A[c][i].y, fma(-vr[i].y, A[c][i].x, ai));
            }
            v32[2 * c] = ar;
            v32[2 * c + 1] = ai;
        }
        double w16[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) w16[t] = swap_sum<32>(v32[t], v32[t + 16]);
        double w8[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) w8[t] = swap_sum<16>(w16[t], w16[t + 8]);
        const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0, h2 = (lane & 2) != 0;
        double w4[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double a0 = w8[t], a1 = w8[t + 4];
            w4[t] = (h8 ? a1 : a0) + dpp_d<0x140>(h8 ? a0 : a1);
        }
        double w2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const double a0 = w4[t], a1 = w4[t + 2];
            w2[t] = (h4 ? a1 : a0) + dpp_d<0x141>(h4 ? a0 : a1);
        }
        double tot = (h2 ? w2[1] : w2[0]) + dpp_d<0x4E>(h2 ? w2[0] : w2[1]);
        tot += dpp_d<0xB1>(tot);
        // Re w_c in lane 4 c, Im w_c in lane 4 c + 2: through LDS to every lane
        if ((lane & 1) == 0) reinterpret_cast<double*>(wsh[wave])[lane >> 1] = tot;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double2 wc = wsh[wave][c];
            const double twx = tauj * wc.x, twy = tauj * wc.y;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {                            // y -= v (tau w)
                const double ax = fma(-vr[i].x, twx, fma(vr[i].y, twy, A[c][i].x));
                const double ay = fma(-vr[i].x, twy, fma(-vr[i].y, twx, A[c][i].y));
                A[c][i] = make_double2(ax, ay);
            }
        }
    }
    // eigenvector of slot c into column act[c] (contiguous)
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int col = 16 * wave + c;
        if (col < cnt) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int row = lane + 64 * i;
                if (row < N) Bm[(long)act[g0 + col] * N + row] = A[c][i];
            }
        }
    }
    }
    __syncthreads();                              // dml and insh are reused by the next group
    }
}

// Subset EVD above 128 frames (padded sizes 160 and 208), steps 1 and 2 of the
// tridiagonal path with the matrix in global memory: the register layout of
// k_heev_tri_reduce would not fit the register file at these sizes. The working
// copy A (column-major, the projector slot of the subset) is reduced column by
// column: the reflector v of column j (one block reduction), p = tau A v over
// the trailing block (thread (g, r): row r, every fourth column from j + 1 + g,
// so each load runs along a column), q = p - (tau / 2)(v^H p) v, and the
// two-sided update A -= v q^H + q v^H of the trailing block. The reflectors go
// where k_heev_tri_vecs reads them (tau in row 0 of v_j, which is zero), the
// tridiagonal form to the same scratch; B (row-major) is left untouched for the
// Jacobi kernel.
template <int N, int RPL>
__global__ void __launch_bounds__(1024) k_heev_big_reduce(Workspace ws) {
    constexpr int NTHR = 1024, NG = NTHR / 256;
    static_assert(N <= 256 && 64 * RPL >= N, "rows per lane of the scan cover the size");
    __shared__ double2 vsh[N], qsh[N];
    __shared__ double2 psum[NG][256];
    __shared__ double dsh[N], esh[N], e2sh[N];
    __shared__ double2 phs[N];
    __shared__ double redd[32];
    __shared__ double bnd[3];
    __shared__ double tau_sh;
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = tid & 255, g = tid >> 8;
    const int nt = ws.sub[s].nt;
    const double2* Bm = ws.bmat + (long)s * N * N;
    double2* A = ws.pmat + (long)s * N * N;                  // working copy, A[c * N + r] = B[r][c]
    double2* H = ws.wvec + (long)s * N * N;
    double* trid = reinterpret_cast<double*>(ws.pmat + (long)s * N * N) + N * N;
    for (int e = tid; e < N * N; e += NTHR) {
        const int c = e / N, rr = e % N;
        A[e] = (rr < nt && c < nt) ? cconj(Bm[(long)c * N + rr]) : make_double2(0.0, 0.0);   // B[rr][c]
    }
    auto block_sum = [&](double v) {
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) redd[wave] = v;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < NTHR / 64; ++w) t += redd[w];
        return t;
    };
    __syncthreads();
    for (int j = 0; j + 2 < nt; ++j) {
        // reflector of column j (rows j + 1 ..)
        const double2 x = (tid > j && tid < nt) ? A[(long)j * N + tid] : make_double2(0.0, 0.0);
        const double s2 = block_sum(tid > j + 1 ? cabs2(x) : 0.0);
        if (tid == j + 1) {
            const double ax0 = sqrt(cabs2(x));
            const double alpha = sqrt(s2 + ax0 * ax0);
            const double2 ph = ax0 > 0.0 ? cscale(x, 1.0 / ax0) : make_double2(1.0, 0.0);
            tau_sh = alpha > 0.0 ? 1.0 / (alpha * (alpha + ax0)) : 0.0;
            vsh[tid] = cadd(x, cscale(ph, alpha));
            phs[j] = cscale(ph, -alpha);                          // complex e_j for now
            dsh[j] = A[(long)j * N + j].x;
        } else if (tid < N) {
            vsh[tid] = tid > j + 1 ? x : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const double tau = tau_sh;
        if (tid < N) H[(long)j * N + tid] = tid == 0 ? make_double2(tau, 0.0) : vsh[tid];
        // p = A v over the trailing block
        double2 acc = make_double2(0.0, 0.0);
        if (r > j && r < nt) {
            for (int c = j + 1 + g; c < nt; c += NG) {
                const double2 a = A[(long)c * N + r], vc = vsh[c];
                acc.x = fma(a.x, vc.x, fma(-a.y, vc.y, acc.x));
                acc.y = fma(a.x, vc.y, fma(a.y, vc.x, acc.y));
            }
        }
        psum[g][r] = acc;
        __syncthreads();
        double2 pr = make_double2(0.0, 0.0), vr = make_double2(0.0, 0.0);
        if (tid < N) {
            for (int gg = 0; gg < NG; ++gg) pr = cadd(pr, psum[gg][tid]);
            pr = cscale(pr, tau);
            vr = vsh[tid];
        }
        const double kr = block_sum(vr.x * pr.x + vr.y * pr.y);   // Re conj(v) p
        const double ki = block_sum(vr.x * pr.y - vr.y * pr.x);   // Im conj(v) p
        if (tid < N) {
            const double2 K = make_double2(0.5 * tau * kr, 0.5 * tau * ki);
            qsh[tid] = csub(pr, cmul(K, vr));
        }
        __syncthreads();
        // A -= v q^H + q v^H on the trailing block
        if (r > j && r < nt) {
            const double2 v_r = vsh[r], q_r = qsh[r];
            for (int c = j + 1 + g; c < nt; c += NG) {
                const double2 vc = vsh[c], qc = qsh[c];
                double2 a = A[(long)c * N + r];
                a.x = fma(-v_r.x, qc.x, fma(-v_r.y, qc.y, a.x));
                a.y = fma(-v_r.y, qc.x, fma(v_r.x, qc.y, a.y));
                a.x = fma(-q_r.x, vc.x, fma(-q_r.y, vc.y, a.x));
                a.y = fma(-q_r.y, vc.x, fma(q_r.x, vc.y, a.y));
                A[(long)c * N + r] = a;
            }
        }
        __syncthreads();
    }
    // last 2 x 2 block
    if (tid == 0 && nt >= 2) {
        dsh[nt - 2] = A[(long)(nt - 2) * N + nt - 2].x;
        dsh[nt - 1] = A[(long)(nt - 1) * N + nt - 1].x;
        phs[nt - 2] = A[(long)(nt - 2) * N + nt - 1];            // row nt - 1, column nt - 2
    }
    if (tid == 0 && nt == 1) dsh[0] = A[0].x;
    __syncthreads();
    // ---- 2. real tridiagonal: |e_j|, the phases D by a prefix product (wave 0,
    // element j in lane j % 64, register j / 64) and the Gershgorin interval
    if (wave == 0) {
        double2 u[RPL];
        double ae[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int j = lane + 64 * i;
            const double2 e = j + 1 < nt ? phs[j] : make_double2(0.0, 0.0);
            ae[i] = sqrt(cabs2(e));
            u[i] = ae[i] > 0.0 ? cscale(e, 1.0 / ae[i]) : make_double2(1.0, 0.0);
            if (j + 1 < nt) {
                esh[j] = ae[i];
                e2sh[j] = ae[i] * ae[i];
            }
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const double2 t = make_double2(__shfl_up(u[i].x, off, 64), __shfl_up(u[i].y, off, 64));
                if (lane >= off) u[i] = cmul(t, u[i]);
            }
        double2 carry = make_double2(1.0, 0.0);
        double lo = 1e300, hi = -1e300, emax = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const double2 incl = cmul(carry, u[i]);
            const double2 prev = make_double2(__shfl_up(incl.x, 1, 64), __shfl_up(incl.y, 1, 64));
            const int j = lane + 64 * i;
            if (j < N) phs[j] = make_double2(lane == 0 ? carry.x : prev.x, lane == 0 ? carry.y : prev.y);
            carry = make_double2(rdl(incl.x, 63), rdl(incl.y, 63));
            const double aup = __shfl_up(ae[i], 1, 64);
            const double aprv = lane == 0 ? (i > 0 ? rdl(ae[i > 0 ? i - 1 : 0], 63) : 0.0) : aup;
            if (j < nt) {
                const double rad = (j > 0 ? aprv : 0.0) + (j + 1 < nt ? ae[i] : 0.0);
                lo = fmin(lo, dsh[j] - rad);
                hi = fmax(hi, dsh[j] + rad);
                if (j + 1 < nt) emax = fmax(emax, ae[i] * ae[i]);
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, m, 64));
            hi = fmax(hi, __shfl_xor(hi, m, 64));
            emax = fmax(emax, __shfl_xor(emax, m, 64));
        }
        if (lane == 0) {
            const double margin = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
            bnd[0] = lo - margin;
            bnd[1] = hi + margin;
            bnd[2] = 1e-290 * fmax(1.0, emax);                        // pivmin
        }
    }
    __syncthreads();
    for (int i = tid; i < N; i += NTHR) {
        trid[i] = dsh[i];
        trid[N + i] = esh[i];
        trid[2 * N + i] = e2sh[i];
        trid[3 * N + i] = phs[i].x;
        trid[4 * N + i] = phs[i].y;
    }
    if (tid == 0) {
        trid[5 * N] = bnd[2];
        trid[5 * N + 1] = bnd[0];
        trid[5 * N + 2] = bnd[1];
    }
}

// Normalise columns, sort by norm descending, write eigenvalues and vectors.
// vout: column-major (vector j contiguous) when col_major, else row-major.
__device__ void jacobi_finish(const double2* G, int nt, int ld, double* lam_out, double2* vout,
                              int ldv, bool col_major) {
    __shared__ double nrm[256];
    __shared__ int rk[256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wave; j < nt; j += nw) {
        double s = 0.0;
        for (int row = lane; row < nt; row += 64) s += cabs2(G[(long)j * ld + row]);
        s = wave_sum(s);
        if (lane == 0) nrm[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nt; j += blockDim.x) {
        int r = 0;
        const double v = nrm[j];
        for (int i = 0; i < nt; ++i) r += (nrm[i] > v) || (nrm[i] == v && i < j);
        rk[j] = r;
        lam_out[r] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nt * nt; e += blockDim.x) {
        const int j = e / nt, row = e % nt;
        const double inv = nrm[j] > 0.0 ? 1.0 / nrm[j] : 0.0;
        const double2 g = cscale(G[(long)j * ld + row], inv);
        const int c = rk[j];
        if (col_major) vout[(long)c * ldv + row] = g;
        else vout[(long)row * ldv + c] = g;
    }
    __syncthreads();
}

// Subset EVD: bmat (row-major Hermitian, stride ntp) -> wvec as column-major
// Jacobi workspace -> sorted eigenvectors back into bmat (column-major).
template <bool IN_LDS>
__global__ void __launch_bounds__(JAC_THREADS) k_jacobi_subsets(Workspace ws, int max_sweeps, int only_flag) {
    extern __shared__ double2 lds_g[];
    const int s = blockIdx.x;
    if (only_flag != 0 && (ws.flags[s] & only_flag) == 0) return;   // not selected: whole block exits
    const int nt = ws.sub[s].nt, ntp = ws.ntp;
    double2* B = ws.bmat + (long)s * ntp * ntp;
    double2* G = IN_LDS ? lds_g : ws.wvec + (long)s * ntp * ntp;
    const int ld = IN_LDS ? nt : ntp;
    for (int e = threadIdx.x; e < nt * nt; e += blockDim.x) {
        const int j = e / nt, row = e % nt;
        G[(long)j * ld + row] = cconj(B[(long)j * ntp + row]);   // column j of B = conj(row j)
    }
    __syncthreads();
    jacobi_core<IN_LDS>(G, nt, ld, max_sweeps, &ws.sweeps[s], &ws.flags[s]);
    jacobi_finish(G, nt, ld, ws.lam + (long)s * ntp, B, ntp, true);
}

// Standalone batched EVD: a (row-major Hermitian [n][nt][nt]) -> w, v (row-major).
template <bool IN_LDS>
__global__ void __launch_bounds__(JAC_THREADS) k_heevd(const double2* a, double* w, double2* v,
                                                       int* sweeps, double2* work, int nt, int max_sweeps,
                                                       int* flags) {
    extern __shared__ double2 lds_g[];
    const int b = blockIdx.x;
    const double2* A = a + (long)b * nt * nt;
    double2* G = IN_LDS ? lds_g : work + (long)b * nt * nt;
    for (int e = threadIdx.x; e < nt * nt; e += blockDim.x) {
        const int j = e / nt, row = e % nt;
        G[(long)j * nt + row] = cconj(A[(long)j * nt + row]);
    }
    __syncthreads();
    jacobi_core<IN_LDS>(G, nt, nt, max_sweeps, &sweeps[b], &flags[b]);
    double2* vo = v ? v + (long)b * nt * nt : nullptr;
    if (vo) {
        jacobi_finish(G, nt, nt, w + (long)b * nt, vo, nt, false);
    } else {
        // eigenvalues only: reuse the workspace slot for the (discarded) vectors
        double2* scratch = work + (long)b * nt * nt;
        if (IN_LDS) jacobi_finish(G, nt, nt, w + (long)b * nt, scratch, nt, false);
        else {
            // G lives in scratch already: compute norms and sort in place of w only
            __shared__ double nrm[256];
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
            for (int j = wave; j < nt; j += nw) {
                double sacc = 0.0;
                for (int row = lane; row < nt; row += 64) sacc += cabs2(G[(long)j * nt + row]);
                sacc = wave_sum(sacc);
                if (lane == 0) nrm[j] = sqrt(sacc);
            }
            __syncthreads();
            for (int j = threadIdx.x; j < nt; j += blockDim.x) {
                int r = 0;
                for (int i = 0; i < nt; ++i) r += (nrm[i] > nrm[j]) || (nrm[i] == nrm[j] && i < j);
                w[(long)b * nt + r] = nrm[j];
            }
        }
    }
}

// ------------------------------------------------------------------ launchers

template <int NTP>
// iarg: subspace iterations (tissue basis) or the keep-R flag (assembly)
static void small_dispatch(const Workspace& ws, int stage, double rho, int iarg, hipStream_t st) {
    if (stage == 0) hipLaunchKernelGGL((k_tissue<NTP>), dim3(ws.S), dim3(256), 0, st, ws, rho, iarg);
    else hipLaunchKernelGGL((k_assemble<NTP>), dim3(ws.S), dim3(AsmCfg<NTP>::NTHR), 0, st, ws, iarg);
}

static hipError_t small_stage(const Workspace& ws, int stage, double rho, int iarg, hipStream_t st) {
    switch (ws.ntp) {
        case 32: small_dispatch<32>(ws, stage, rho, iarg, st); break;
        case 64: small_dispatch<64>(ws, stage, rho, iarg, st); break;
        case 96: small_dispatch<96>(ws, stage, rho, iarg, st); break;
        case 128: small_dispatch<128>(ws, stage, rho, iarg, st); break;
        case 160: small_dispatch<160>(ws, stage, rho, iarg, st); break;
        case 208: small_dispatch<208>(ws, stage, rho, iarg, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_windows(const Workspace& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_windows, dim3(ws.S), dim3(256), 0, st, ws);
    return hipGetLastError();
}

hipError_t launch_tissue(const Workspace& ws, double rho, int iters, hipStream_t st) {
    return small_stage(ws, 0, rho, iters, st);
}

hipError_t launch_assemble(const Workspace& ws, int keep_r, hipStream_t st) {
    return small_stage(ws, 1, 0.0, keep_r ? 1 : 0, st);
}

// The tridiagonal solver and its vector stage hold B padded to 16 columns per
// wave and address every per-subset slot with that size: up to 128 frames the
// class must be one of those sizes.
static bool tri_sized(int ntp) { return ntp > 128 || ntp == 32 || ntp == 64 || ntp == 96 || ntp == 128; }

// The Jacobi solver for the subsets selected by sel (0: every subset; the
// fallback flag: those the eigenvector kernel handed back).
static void launch_jacobi(const Workspace& ws, int max_sweeps, int nt_max, int sel, hipStream_t st) {
    if (ws.ntp <= 32) hipLaunchKernelGGL((k_jacobi_reg<1, 2>), dim3(ws.S), dim3(128), 0, st, ws, max_sweeps, sel);
    else if (ws.ntp <= 64) hipLaunchKernelGGL((k_jacobi_reg<1, 4>), dim3(ws.S), dim3(256), 0, st, ws, max_sweeps, sel);
    else if (ws.ntp == 96) hipLaunchKernelGGL((k_jacobi_reg<2, 6>), dim3(ws.S), dim3(384), 0, st, ws, max_sweeps, sel);
    else if (ws.ntp <= 128) hipLaunchKernelGGL((k_jacobi_reg<2, 8>), dim3(ws.S), dim3(512), 0, st, ws, max_sweeps, sel);
    else if (nt_max <= JAC_LDS_NT) {
        const size_t lds = (size_t)nt_max * nt_max * sizeof(double2);
        hipLaunchKernelGGL((k_jacobi_subsets<true>), dim3(ws.S), dim3(JAC_THREADS), lds, st, ws, max_sweeps, sel);
    } else {
        hipLaunchKernelGGL((k_jacobi_subsets<false>), dim3(ws.S), dim3(JAC_THREADS), 0, st, ws, max_sweeps, sel);
    }
}

// Eigenvalues: the tridiagonal path (method 0; register-resident reduction up
// to 128 frames, global-memory reduction above, then the multisection), or the
// Jacobi solver for every subset (method 1), which also forms the vectors.
hipError_t launch_evd(const Workspace& ws, int max_sweeps, int nt_max, int method, hipStream_t st) {
    if (!tri_sized(ws.ntp)) return hipErrorInvalidValue;
    if (method != 0) {
        launch_jacobi(ws, max_sweeps, nt_max, 0, st);
        return hipGetLastError();
    }
    switch (ws.ntp) {
        case 32:
            hipLaunchKernelGGL((k_heev_tri_reduce<1, 2>), dim3(ws.S), dim3(128), 0, st, ws);
            hipLaunchKernelGGL((k_heev_sturm<32, 128>), dim3(ws.S), dim3(128), 0, st, ws);
            break;
        case 64:
            hipLaunchKernelGGL((k_heev_tri_reduce<1, 4>), dim3(ws.S), dim3(256), 0, st, ws);
            hipLaunchKernelGGL((k_heev_sturm<64, 256>), dim3(ws.S), dim3(256), 0, st, ws);
            break;
        case 96:
            hipLaunchKernelGGL((k_heev_tri_reduce<2, 6>), dim3(ws.S), dim3(384), 0, st, ws);
            hipLaunchKernelGGL((k_heev_sturm<96, 384>), dim3(ws.S), dim3(384), 0, st, ws);
            break;
        case 128:
            hipLaunchKernelGGL((k_heev_tri_reduce<2, 8>), dim3(ws.S), dim3(512), 0, st, ws);
            hipLaunchKernelGGL((k_heev_sturm<128, 512>), dim3(ws.S), dim3(512), 0, st, ws);
            break;
        case 160:
            hipLaunchKernelGGL((k_heev_big_reduce<160, 3>), dim3(ws.S), dim3(1024), 0, st, ws);
            hipLaunchKernelGGL((k_heev_sturm<160, 1024>), dim3(ws.S), dim3(1024), 0, st, ws);
            break;
        default:
            hipLaunchKernelGGL((k_heev_big_reduce<208, 4>), dim3(ws.S), dim3(1024), 0, st, ws);
            hipLaunchKernelGGL((k_heev_sturm<208, 1024>), dim3(ws.S), dim3(1024), 0, st, ws);
            break;
    }
    return hipGetLastError();
}

// Eigenvectors after the weights are known (tridiagonal path, at every size;
// all = 1 forms every component's, as the NCC rule needs), then the Jacobi
// solver for the subsets whose selected components sit in a near-degenerate
// pair; the Jacobi path (method 1) produced its vectors already.
hipError_t launch_evd_vectors(const Workspace& ws, int method, int all, int max_sweeps, int nt_max, hipStream_t st) {
    if (!tri_sized(ws.ntp)) return hipErrorInvalidValue;
    if (method != 0) return hipSuccess;
    if (ws.ntp == 160) hipLaunchKernelGGL((k_heev_tri_vecs<3, 10>), dim3(ws.S), dim3(256), 0, st, ws, all);
    else if (ws.ntp == 208) hipLaunchKernelGGL((k_heev_tri_vecs<4, 13>), dim3(ws.S), dim3(256), 0, st, ws, all);
    else if (ws.ntp <= 32) hipLaunchKernelGGL((k_heev_tri_vecs<1, 2>), dim3(ws.S), dim3(128), 0, st, ws, all);
    else if (ws.ntp <= 64) hipLaunchKernelGGL((k_heev_tri_vecs<1, 4>), dim3(ws.S), dim3(256), 0, st, ws, all);
    else if (ws.ntp == 96) hipLaunchKernelGGL((k_heev_tri_vecs<2, 6>), dim3(ws.S), dim3(256), 0, st, ws, all);
    else hipLaunchKernelGGL((k_heev_tri_vecs<2, 8>), dim3(ws.S), dim3(256), 0, st, ws, all);
    launch_jacobi(ws, max_sweeps, nt_max, FLAG_EVD_FALLBACK, st);
    return hipGetLastError();
}

hipError_t launch_heevd(int n, int nt, const double2* a, double* w, double2* v, int* sweeps, double2* work,
                        int max_sweeps, int* flags, hipStream_t st) {
    if (nt <= JAC_LDS_NT) {
        const size_t lds = (size_t)nt * nt * sizeof(double2);
        hipLaunchKernelGGL((k_heevd<true>), dim3(n), dim3(JAC_THREADS), lds, st, a, w, v, sweeps, work, nt,
                           max_sweeps, flags);
    } else {
        hipLaunchKernelGGL((k_heevd<false>), dim3(n), dim3(JAC_THREADS), 0, st, a, w, v, sweeps, work, nt,
                           max_sweeps, flags);
    }
    return hipGetLastError();
}

}  // namespace lcf
