// Internal types and device helpers of the localized EVD clutter filter library.
// Shared by the host runtime (runtime.hip) and the kernel files (k_*.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcf {

// Tissue deflation: at most RMAX leading eigen-directions are split off in FP64
// (the rank-r part of the covariance and of the projection). REXT is RMAX padded
// to one 16-wide MFMA tile; those columns extend the Gram of the deflated data.
constexpr int RMAX = 8;
constexpr int REXT = 16;
// Pixels per LDS batch in the Gram and reprojection kernels.
constexpr int PIX = 32;
// Reprojection tiles are TW pixels wide (one MFMA row tile per image row) and
// 2 or 4 rows high: 4 only up to 128 frames (the accumulators of wider subsets
// fill the register file). Chosen per launch group (default, or by the autotuner).
constexpr int TW = 16;
constexpr int TROWS = 4;
__host__ __device__ constexpr int trows_max(int ntp) { return ntp <= 128 ? 4 : 2; }
// Pixels per Gram work item (split-K chunk); several LDS batches each.
constexpr int CHUNK = 1024;

// One window subset of one packet (Eq. 11 / Fig. 3).
struct SubsetDesc {
    const float2* iq;   // packet base, complex64 [nt][ny][nx]
    int ny, nx, nt;
    int pkt;            // packet index within the call
    int d;              // subset index within the packet (a*gx + b)
    int y0, y1, x0, x1; // inclusive box of non-zero window values
    int bw, neff;       // box width, box pixel count
    int flat;           // 1 = flat window (w = 1 inside the box)
    int wy_off, wx_off; // offsets of the 1-D FP64 window factors in the table pool
    double cy, cx, sy, sx;
    double npix_nt;     // Npix * Nt of the packet (Eq. 13 normalisation)
    long ew_off;        // offset of this subset's caller-given weights in explicit_w (floats)
};

// A split-K chunk of a subset's box pixels [q0, q1) in box row-major order.
struct ChunkDesc {
    int s;      // subset index in the launch
    int q0, q1;
};

// A reprojection tile: rows y .. y + nrow - 1 (nrow <= the group's trows), columns [x0, x1]
// of packet pkt, covered by the subsets cover[cov_off .. cov_off + cov_cnt)
// (ascending subset order).
struct TileDesc {
    int pkt, y, x0, x1;
    int nrow;
    int cov_off, cov_cnt;
};

struct PacketDesc {
    const float2* iq;
    float* iq_out;      // interleaved complex64 as floats, may be null
    float* pd;
    int ny, nx, nt;
    int pd_mode;
};

// Device workspace of one launch group (all subsets share the padded size ntp).
struct Workspace {
    int S;              // subsets
    int ntp;            // padded Nt (multiple of 16)
    int nte;            // ntp + REXT
    const SubsetDesc* sub;
    const ChunkDesc* chunks;
    int nchunks;
    const int* chunk_begin;   // [S+1] first chunk of each subset
    const TileDesc* tiles;
    int ntiles;
    int trows;          // rows per reprojection tile (2 or 4)
    int rvar;           // reprojection kernel: 0 = every wave does everything, 1 = producer/consumer waves
    const int* cover;
    const PacketDesc* pkts;
    double* wtab;       // window factor pool
    float* partial;     // Gram partials [nchunks][ntile_pairs*2][256]
    float2* rwin;       // [S][ntp][ntp] windowed covariance of pass 1, FP32 (it only locates the
                        // tissue subspace, and its own Gram is no more accurate than that)
    double2* rext;      // [S][nte][nte] Gram of [C' | Y] (pass 2)
    double2* hv;        // [S][RMAX][ntp] Householder vectors
    double* htau;       // [S][RMAX]
    double2* vr64;      // [S][ntp][RMAX] tissue basis V_r (FP64)
    float2* vr32;       // [S][ntp][RMAX] V_r rounded to FP32
    int* rank;          // [S]
    double2* bmat;      // [S][ntp][ntp] B = Q^H R Q, then Jacobi workspace
    double2* wvec;      // [S][ntp][ntp] eigenvectors of B (row-major, column j = vector j)
    double* lam;        // [S][ntp]
    double* wts;        // [S][ntp] eigencomponent weights
    int* kcut;          // [S]
    int* flags;         // [S]
    int* sweeps;        // [S]
    double* alpha;      // [S]
    double* curve;      // [S][ntp] Eq. 8 curve of the NCC rule (NaN where it has no value)
    double2* pmat;      // [S][ntp][ntp] projector P in the original basis (FP64)
    float* breal;       // [S][2*nte][2*ntp] real form of [P; M] for the reprojection
    const float* explicit_w;   // [S][nt] caller weights (EXPLICIT)
};

// ------------------------------------------------------------------ helpers

typedef __bf16 lcf_bf16x2 __attribute__((ext_vector_type(2)));
typedef float lcf_floatx2 __attribute__((ext_vector_type(2)));

// Split-BF16 pair: (re, im) = hi + lo with hi = bf16(x), lo = bf16(x - hi), both
// rounded to nearest even by the packed hardware conversion. Each word holds
// the re part in its low half and the im part in its high half.
__device__ __forceinline__ void split_bf16x2(float re, float im, uint32_t& h, uint32_t& l) {
    const lcf_floatx2 v = {re, im};
    h = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, lcf_bf16x2));
    const lcf_floatx2 r = {re - __uint_as_float(h << 16), im - __uint_as_float(h & 0xFFFF0000u)};
    l = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, lcf_bf16x2));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// acc + a b and acc + conj(a) b, each component as two fused multiply-adds
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
__device__ __forceinline__ double2 cfmac(double2 a, double2 b, double2 acc) {
    return make_double2(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// A double read from one lane (two scalar reads).
__device__ __forceinline__ double rdl(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Lane-swap sum of two wave-wide doubles: for M = 32 lanes below 32 return
// a[l] + a[l + 32] and lanes above 32 return b[l - 32] + b[l]; for M = 16 the
// same within each 32-lane half (rows of 16 lanes), a in even rows, b in odd.
template <int M>
__device__ __forceinline__ double swap_sum(double a, double b) {
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
    const double p = __longlong_as_double((long long)(((unsigned long long)x1 << 32) | x0));
    const double q = __longlong_as_double((long long)(((unsigned long long)y1 << 32) | y0));
    return p + q;
}

// Data-parallel lane moves of a double within a row of 16 lanes (DPP):
// 0xB1 = quad_perm [1,0,3,2] (lane ^ 1), 0x4E = quad_perm [2,3,0,1] (lane ^ 2),
// 0x141 = row_half_mirror (lane ^ 7), 0x140 = row_mirror (lane ^ 15).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Sum of a double over the 64 lanes, every lane getting the same bits: lane
// moves within rows of 16 (DPP), then the row-swap instructions.
__device__ __forceinline__ double wave_sum_x(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    v = swap_sum<16>(v, v);
    return swap_sum<32>(v, v);
}

// block_sum / block_sum2 with the lane-move reduction inside each wave (every
// thread of the block must take part).
__device__ __forceinline__ double block_sum_x(double v, double* red) {
    v = wave_sum_x(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ double2 block_sum2_x(double2 v, double* red) {
    v.x = wave_sum_x(v.x);
    v.y = wave_sum_x(v.y);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[2 * w] = v.x; red[2 * w + 1] = v.y; }
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < nw; ++i) { s.x += red[2 * i]; s.y += red[2 * i + 1]; }
    return s;
}

// Block-wide sum of a double over blockDim.x threads (multiple of 64); red is
// __shared__ scratch of at least blockDim.x/64 doubles. All threads get the sum.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ double2 block_sum2(double2 v, double* red) {
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[2 * w] = v.x; red[2 * w + 1] = v.y; }
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < nw; ++i) { s.x += red[2 * i]; s.y += red[2 * i + 1]; }
    return s;
}

}  // namespace lcf
