// Host runtime of the localized EVD clutter filter: argument validation, window
// geometry and work lists (plans), the device scratch arena, launch schedules
// (batched or the paper's sequential per-subset loop), optional hipGraph replay,
// and the C ABI declared in include/lcf.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lcf.h"
#include "lcf_internal.h"
#include "lcf_kernels.h"

using namespace lcf;

// Fixed device block of the allocation-free entry point (lcf_filter_noalloc):
// descriptors, workspace and network activations of one call. Each device the
// library runs on holds its own copy until the process ends. In host code this
// name is only a stand-in for the symbol: its device address is taken once per
// device with hipGetSymbolAddress (lcf_create) and only that address is used.
static __device__ __align__(256) unsigned char scratch[LCF_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device -> address of `scratch` on that device

// Called with `device` current: look up (once per device) the address of the
// fixed block there.
lcf_status init_scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return LCF_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return LCF_ERR_DEVICE;
    g_scratch_ptr[device] = (char*)ptr;
    return LCF_OK;
}

char* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// Padded frame classes. Up to 128 frames they are exactly the sizes of the
// tridiagonal EVD's 2-, 4-, 6- and 8-wave shapes (16 columns per wave), which
// hold B at that size and address it with it.
const int NTP_CLASSES[] = {32, 64, 96, 128, 160, 208};
constexpr int NT_MAX = 208;

int ntp_class(int nt) {
    for (int c : NTP_CLASSES)
        if (nt <= c) return c;
    return -1;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Window {
    double cy, cx, sy, sx;
    int y0, y1, x0, x1;
    bool flat;
};

// Window grid of Eq. 11 / Fig. 3 (same formulas as the reference definition):
// centre (j + 1/2) * spacing - 1/2, sigma = sigma_frac * spacing, box of
// +-trunc_sigmas * sigma clipped to the image; flat window for sigma_frac == 0.
std::vector<Window> make_windows(const lcf_geometry& g) {
    std::vector<Window> out;
    const double dy = (double)g.ny / g.gy, dx = (double)g.nx / g.gx;
    for (int a = 0; a < g.gy; ++a)
        for (int b = 0; b < g.gx; ++b) {
            Window w;
            w.cy = (a + 0.5) * dy - 0.5;
            w.cx = (b + 0.5) * dx - 0.5;
            w.sy = g.sigma_frac * dy;
            w.sx = g.sigma_frac * dx;
            w.flat = g.sigma_frac == 0.0;
            if (w.flat || g.trunc_sigmas == 0.0) {
                w.y0 = 0; w.y1 = g.ny - 1; w.x0 = 0; w.x1 = g.nx - 1;
            } else {
                w.y0 = std::max(0, (int)std::ceil(w.cy - g.trunc_sigmas * w.sy));
                w.y1 = std::min(g.ny - 1, (int)std::floor(w.cy + g.trunc_sigmas * w.sy));
                w.x0 = std::max(0, (int)std::ceil(w.cx - g.trunc_sigmas * w.sx));
                w.x1 = std::min(g.nx - 1, (int)std::floor(w.cx + g.trunc_sigmas * w.sx));
            }
            out.push_back(w);
        }
    return out;
}

lcf_status validate_geometry(const lcf_geometry* g) {
    if (!g) return LCF_ERR_INVALID_ARG;
    if (g->ny < 1 || g->nx < 1 || g->nt < 4 || g->gy < 1 || g->gx < 1) return LCF_ERR_INVALID_ARG;
    if (g->gy > g->ny || g->gx > g->nx || g->reserved != 0) return LCF_ERR_INVALID_ARG;
    if (!(g->sigma_frac >= 0.0) || !(g->trunc_sigmas >= 0.0) || !std::isfinite(g->sigma_frac) ||
        !std::isfinite(g->trunc_sigmas))
        return LCF_ERR_INVALID_ARG;
    if (g->sigma_frac == 0.0 && (g->gy != 1 || g->gx != 1)) return LCF_ERR_INVALID_ARG;
    if ((long)g->ny * g->nx > (1L << 26)) return LCF_ERR_UNSUPPORTED;
    if (g->nt > NT_MAX) return LCF_ERR_UNSUPPORTED;
    return LCF_OK;
}

lcf_status validate_threshold(const lcf_threshold* t, int nt) {
    if (!t) return LCF_ERR_INVALID_ARG;
    if (t->cut < 0 || t->cut > 7 || t->shape < 0 || t->shape > 1 || t->pd_mode < 0 || t->pd_mode > 2)
        return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_FIXED_K && (t->k_fixed < 0 || t->k_fixed > nt)) return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_KNEE && (!(t->beta_knee > 0.0) || !(t->knee_max_frac > 0.0) || t->knee_max_frac > 1.0))
        return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_MEDIAN && !(t->beta_median > 0.0 && std::isfinite(t->beta_median)))
        return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_SLOPE && !(t->slope_thr > 0.0 && std::isfinite(t->slope_thr)))
        return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_POWER && !(t->beta_power > 0.0 && std::isfinite(t->beta_power)))
        return LCF_ERR_INVALID_ARG;
    if (t->shape == LCF_SHAPE_SIGMOID && (t->cut <= LCF_CUT_KNEE || t->cut == LCF_CUT_MEDIAN ||
                                          t->cut == LCF_CUT_SLOPE || t->cut == LCF_CUT_NCC) &&
        !(t->beta_sigmoid > 0.0))
        return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_EXPLICIT && t->explicit_w == nullptr) return LCF_ERR_INVALID_ARG;
    if (!(t->deflate_rho >= 0.0) || t->deflate_rho >= 1.0) return LCF_ERR_INVALID_ARG;
    if (t->cut == LCF_CUT_MLP && (!(t->beta_knee > 0.0) || !(t->knee_max_frac > 0.0) ||
                                  t->knee_max_frac > 1.0 || !(t->beta_sigmoid > 0.0)))
        return LCF_ERR_INVALID_ARG;
    return LCF_OK;
}

lcf_status validate_precision(int p) {
    if (p == LCF_PREC_FP32 || p == LCF_PREC_BF16X3) return LCF_OK;
    return LCF_ERR_INVALID_ARG;
}

struct TuneChoice {
    int chunk;      // split-K chunk of the Gram passes (box pixels)
    int trows;      // image rows per reprojection tile
    int rvar;       // reprojection kernel variant
    int evd;        // subset EVD up to 128 frames: 0 tridiagonal, 1 Jacobi; -1 the context's
};

struct PacketIn {
    lcf_geometry g;
    const void* iq;
    void* iq_out;
    float* pd;
    long ew_off;    // first caller-given weight of this packet in explicit_w (floats)
};

// Host-side plan of one launch group (packets sharing the padded Nt class).
struct Plan {
    int ntp = 0, nt_max = 0;
    int chunk = CHUNK;      // split-K chunk of the Gram passes (box pixels)
    int trows = 2;          // image rows per reprojection tile (2 or 4)
    int rvar = 0;           // reprojection kernel variant (1: producer/consumer, FP32 with 4-row tiles only)
    int evd = -1;           // subset EVD method (LCF_OPT_EVD values); -1 the context's
    std::vector<SubsetDesc> sub;
    std::vector<ChunkDesc> chunks;
    std::vector<int> chunk_begin;
    std::vector<TileDesc> tiles;
    std::vector<int> cover;
    std::vector<PacketDesc> pkts;
    std::vector<int> pkt_first_subset;
    size_t wtab_len = 0;
};

void build_plan(Plan& pl, const std::vector<PacketIn>& in, const std::vector<int>& idx, int pd_mode, int chunk,
                int trows, int rvar) {
    pl.ntp = 0;
    pl.nt_max = 0;
    pl.chunk = chunk;
    pl.trows = trows;
    pl.rvar = (trows == 4) ? rvar : 0;
    for (int i : idx) {
        pl.ntp = std::max(pl.ntp, ntp_class(in[i].g.nt));
        pl.nt_max = std::max(pl.nt_max, in[i].g.nt);
    }
    int wtab = 0;
    for (size_t pi = 0; pi < idx.size(); ++pi) {
        const PacketIn& p = in[idx[pi]];
        const lcf_geometry& g = p.g;
        PacketDesc pd;
        pd.iq = (const float2*)p.iq;
        pd.iq_out = (float*)p.iq_out;
        pd.pd = p.pd;
        pd.ny = g.ny; pd.nx = g.nx; pd.nt = g.nt;
        pd.pd_mode = pd_mode;
        pl.pkts.push_back(pd);
        const int first = (int)pl.sub.size();
        pl.pkt_first_subset.push_back(first);
        const std::vector<Window> wins = make_windows(g);
        for (size_t d = 0; d < wins.size(); ++d) {
            const Window& w = wins[d];
            SubsetDesc s;
            s.iq = (const float2*)p.iq;
            s.ny = g.ny; s.nx = g.nx; s.nt = g.nt;
            s.pkt = (int)pi;
            s.d = (int)d;
            s.y0 = w.y0; s.y1 = w.y1; s.x0 = w.x0; s.x1 = w.x1;
            s.bw = w.x1 - w.x0 + 1;
            s.neff = (w.y1 - w.y0 + 1) * s.bw;
            s.flat = w.flat ? 1 : 0;
            s.cy = w.cy; s.cx = w.cx; s.sy = w.sy; s.sx = w.sx;
            s.wy_off = wtab;
            wtab += w.y1 - w.y0 + 1;
            s.wx_off = wtab;
            wtab += s.bw;
            s.npix_nt = (double)g.ny * g.nx * g.nt;
            s.ew_off = p.ew_off + (long)d * g.nt;
            const int sidx = (int)pl.sub.size();
            pl.chunk_begin.push_back((int)pl.chunks.size());
            for (int q = 0; q < s.neff; q += pl.chunk)
                pl.chunks.push_back(ChunkDesc{sidx, q, std::min(s.neff, q + pl.chunk)});
            pl.sub.push_back(s);
        }
        // Reprojection tiles of trows rows x TW pixels with their covering subsets.
        // The tile origin is shifted (per axis, 0..size-1) so that as few box
        // edges as possible fall inside tiles: with grid windows a tile's
        // covering count is (#window rows over its rows) x (#window columns
        // over its columns), so each axis is chosen on its own.
        const int last = (int)pl.sub.size();
        const int trows = pl.trows;
        auto best_origin = [&](int n, int size, int ngrid, int stride, bool xaxis) {
            int best = 0;
            long best_cost = -1;
            for (int o = 0; o < size; ++o) {
                long cost = 0;
                for (int a0 = o - size; a0 < n; a0 += size) {
                    const int lo = std::max(0, a0), hi = std::min(n - 1, a0 + size - 1);
                    if (lo > hi) continue;
                    for (int j = 0; j < ngrid; ++j) {
                        const SubsetDesc& sd = pl.sub[first + j * stride];
                        const int b0 = xaxis ? sd.x0 : sd.y0, b1 = xaxis ? sd.x1 : sd.y1;
                        cost += (hi >= b0 && lo <= b1);
                    }
                }
                if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = o; }
            }
            return best;
        };
        const int ox = best_origin(g.nx, TW, g.gx, 1, true);
        const int oy = best_origin(g.ny, trows, g.gy, g.gx, false);
        // Tiles are listed patch by patch (patches of 64 rows x 32 pixels, tiles
        // row-major inside): the work-groups of one XCD run consecutive tiles, and
        // a compact patch shares more covering subsets, so more [P; M] operands
        // stay in that XCD's L2.
        const int pr = std::max(1, 64 / trows), pc = std::max(1, 32 / TW);
        std::vector<std::pair<long, TileDesc>> ptiles;
        int iy = -1;
        for (int ys = oy - trows; ys < g.ny; ys += trows) {
            const int ty0 = std::max(0, ys), ty1 = std::min(g.ny - 1, ys + trows - 1);
            if (ty0 > ty1) continue;
            ++iy;
            int ix = -1;
            for (int xs = ox - TW; xs < g.nx; xs += TW) {
                const int tx0 = std::max(0, xs), tx1 = std::min(g.nx - 1, xs + TW - 1);
                if (tx0 > tx1) continue;
                ++ix;
                TileDesc t;
                t.pkt = (int)pi;
                t.y = ty0;
                t.nrow = ty1 - ty0 + 1;
                t.x0 = tx0;
                t.x1 = tx1;
                t.cov_off = (int)pl.cover.size();
                for (int s = first; s < last; ++s) {
                    const SubsetDesc& sd = pl.sub[s];
                    if (ty1 >= sd.y0 && ty0 <= sd.y1 && tx1 >= sd.x0 && tx0 <= sd.x1) pl.cover.push_back(s);
                }
                t.cov_cnt = (int)pl.cover.size() - t.cov_off;
                const long patch = (long)(iy / pr) * 1000000L + ix / pc;
                ptiles.push_back({(patch * pr + iy % pr) * pc + ix % pc, t});
            }
        }
        std::stable_sort(ptiles.begin(), ptiles.end(),
                         [](const std::pair<long, TileDesc>& a, const std::pair<long, TileDesc>& b) { return a.first < b.first; });
        for (const auto& pt : ptiles) pl.tiles.push_back(pt.second);
    }
    pl.chunk_begin.push_back((int)pl.chunks.size());
    pl.wtab_len = (size_t)wtab;
}

}  // namespace

struct lcf_stream {
    lcf_context* ctx = nullptr;
    lcf_geometry geo{};
    lcf_threshold thr{};
    int prec = 0;
    Plan plan;
    double2* rbuf[2] = {nullptr, nullptr};   // FP64 covariance of the last packet / the next one
    double2* part = nullptr;                 // band partials of the new columns
    int cur = 0;                             // rbuf[cur] holds the last packet's covariance
    bool primed = false;
};

struct lcf_context {
    int device = 0;
    int schedule = 0;
    int max_sweeps = 30;
    int use_graph = 0;
    int sub_iters = 3;
    char* dbuf = nullptr;
    size_t dcap = 0;
    char* hbuf = nullptr;
    size_t hcap = 0;
    hipEvent_t staged = nullptr;   // host staging buffer free again once this completes
    bool staged_pending = false;
    int* sticky = nullptr;         // device: OR of all per-subset flags since lcf_sync
    // graph cache: signature -> executable graph
    std::map<std::string, hipGraphExec_t> graphs;
    // per-stage event timing
    int timing = 0;
    std::vector<hipEvent_t> evpool;
    size_t evnext = 0;
    std::vector<std::pair<int, size_t>> evpending;   // (stage, index of start event)
    double stage_ms[LCF_NUM_STAGES] = {0};
    long long stage_n[LCF_NUM_STAGES] = {0};
    int evd_method = 0;            // 0: tridiagonal solver (Jacobi for flagged subsets), 1: Jacobi
    long mlp_gate_mdb = 100;       // learned weights: gate threshold in milli-dB, < 0 = no gate
    // autotuner: choices per launch-group class (tune_key)
    int autotune = 0;
    std::map<std::string, TuneChoice> tuned;
    // learned weights
    MlpDev mlp{};
    bool mlp_ready = false;
    long long mlp_step = 0;
    float* mlp_scratch = nullptr;
    size_t mlp_scratch_cap = 0;     // floats
    // allocation-free entry point: pageable host staging of its plan uploads,
    // free again once fixed_staged completes
    std::vector<char> fixed_host;
    hipEvent_t fixed_staged = nullptr;
    bool fixed_pending = false;
};

namespace {

lcf_status ensure_device(lcf_context* c, size_t bytes) {
    if (bytes <= c->dcap) return LCF_OK;
    if (c->dbuf) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(c->dbuf) != hipSuccess) return LCF_ERR_DEVICE;
        c->dbuf = nullptr;
        c->dcap = 0;
        // the graphs hold addresses in the old block; a failed destroy leaves nothing to undo
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
    }
    const size_t want = align_up(bytes + bytes / 4, 1 << 20);
    if (hipMalloc((void**)&c->dbuf, want) != hipSuccess) { c->dbuf = nullptr; return LCF_ERR_OUT_OF_MEMORY; }
    c->dcap = want;
    return LCF_OK;
}

lcf_status ensure_host(lcf_context* c, size_t bytes) {
    if (c->staged_pending) {
        if (hipEventSynchronize(c->staged) != hipSuccess) return LCF_ERR_DEVICE;
        c->staged_pending = false;
    }
    if (bytes <= c->hcap) return LCF_OK;
    if (c->hbuf) {
        if (hipHostFree(c->hbuf) != hipSuccess) return LCF_ERR_DEVICE;
        c->hbuf = nullptr;
        c->hcap = 0;
    }
    const size_t want = align_up(bytes + bytes / 4, 1 << 16);
    if (hipHostMalloc((void**)&c->hbuf, want, hipHostMallocDefault) != hipSuccess) {
        c->hbuf = nullptr;
        c->hcap = 0;
        return LCF_ERR_OUT_OF_MEMORY;
    }
    c->hcap = want;
    return LCF_OK;
}

// LCF_ERR_UNSUPPORTED when `st` is being captured into a graph by the caller
// (the entry points that stage plans or grow buffers cannot be captured).
lcf_status refuse_capture(hipStream_t st) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (st != nullptr && hipStreamIsCapturing(st, &cap) != hipSuccess) return LCF_ERR_DEVICE;
    return cap == hipStreamCaptureStatusNone ? LCF_OK : LCF_ERR_UNSUPPORTED;
}

void drop_graphs(lcf_context* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);   // nothing to undo on failure
    c->graphs.clear();
}

// Everything that shapes a launch group's kernels and their arguments, except
// the packet pointers (those live in the descriptors re-uploaded every call).
std::string graph_key(lcf_context* c, const Plan& pl, const std::vector<PacketIn>& in,
                      const std::vector<int>& idx, const lcf_threshold* thr, int prec, const lcf_diag* diag) {
    std::string k;
    char buf[256];
    for (int i : idx) {
        const lcf_geometry& g = in[i].g;
        std::snprintf(buf, sizeof buf, "g%d,%d,%d,%d,%d,%.17g,%.17g,%d|", g.ny, g.nx, g.nt, g.gy, g.gx, g.sigma_frac,
                      g.trunc_sigmas, in[i].iq_out != nullptr);
        k += buf;
    }
    std::snprintf(buf, sizeof buf, "t%d,%d,%d,%d,%.17g,%.17g,%.17g,%.17g,%p|p%d,s%d,w%d,i%d,n%d", thr->cut, thr->shape,
                  thr->pd_mode, thr->k_fixed, thr->beta_knee, thr->knee_max_frac, thr->beta_sigmoid, thr->deflate_rho,
                  (const void*)thr->explicit_w, prec, c->schedule, c->max_sweeps, c->sub_iters, pl.ntp);
    k += buf;
    std::snprintf(buf, sizeof buf, "|m%.17g,%.17g,%.17g", thr->beta_median, thr->slope_thr, thr->beta_power);
    k += buf;
    std::snprintf(buf, sizeof buf, "|c%d,r%d,v%d,e%d,g%ld", pl.chunk, pl.trows, pl.rvar,
                  pl.evd >= 0 ? pl.evd : c->evd_method, c->mlp_gate_mdb);
    k += buf;
    if (diag) {
        std::snprintf(buf, sizeof buf, "|d%p,%p,%p,%p,%p,%p,%p,%p,%p,%p,%p", (void*)diag->eigvals,
                      (void*)diag->weights, (void*)diag->k, (void*)diag->sweeps, (void*)diag->flags,
                      (void*)diag->alpha, (void*)diag->cov, (void*)diag->eigvecs, (void*)diag->rank,
                      (void*)diag->curve, (void*)diag->mlp_gate);
        k += buf;
    }
    return k;
}

lcf_status ensure_mlp_scratch(lcf_context* c, size_t floats) {
    if (floats <= c->mlp_scratch_cap) return LCF_OK;
    drop_graphs(c);
    if (c->mlp_scratch) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(c->mlp_scratch) != hipSuccess) return LCF_ERR_DEVICE;
        c->mlp_scratch = nullptr;
        c->mlp_scratch_cap = 0;
    }
    const size_t want = align_up(floats + floats / 4, 1 << 16);
    if (hipMalloc((void**)&c->mlp_scratch, want * sizeof(float)) != hipSuccess) return LCF_ERR_OUT_OF_MEMORY;
    c->mlp_scratch_cap = want;
    return LCF_OK;
}

lcf_status ensure_mlp(lcf_context* c) {
    if (c->mlp.master) return LCF_OK;
    const size_t n = MLP_NPARAM;
    if (hipMalloc((void**)&c->mlp.master, n * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&c->mlp.wbf, n * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc((void**)&c->mlp.m, n * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&c->mlp.v, n * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&c->mlp.grad, n * sizeof(float)) != hipSuccess)
        return LCF_ERR_OUT_OF_MEMORY;
    if (hipMemset(c->mlp.m, 0, n * sizeof(float)) != hipSuccess ||
        hipMemset(c->mlp.v, 0, n * sizeof(float)) != hipSuccess ||
        hipMemset(c->mlp.grad, 0, n * sizeof(float)) != hipSuccess)
        return LCF_ERR_DEVICE;
    return LCF_OK;
}

uint32_t crc32_update(uint32_t crc, const void* data, size_t len) {
    static uint32_t table[256];
    static bool init = false;
    if (!init) {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            table[i] = c;
        }
        init = true;
    }
    const unsigned char* p = (const unsigned char*)data;
    crc = ~crc;
    for (size_t i = 0; i < len; ++i) crc = table[(crc ^ p[i]) & 0xFF] ^ (crc >> 8);
    return ~crc;
}

struct Layout {
    size_t off_sub, off_chunks, off_cbeg, off_tiles, off_cover, off_pkts, host_bytes;
    size_t off_wtab, off_partial, off_rwin, off_rext, off_hv, off_htau, off_vr64, off_vr32, off_rank, off_bmat,
        off_wvec, off_lam, off_wts, off_kcut, off_flags, off_sweeps, off_alpha, off_curve, off_pmat, off_breal, total;
};

Layout make_layout(const Plan& pl) {
    Layout L;
    const size_t S = pl.sub.size(), ntp = pl.ntp, nte = ntp + REXT;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align_up(o + bytes, 256); return r; };
    L.off_sub = take(S * sizeof(SubsetDesc));
    L.off_chunks = take(pl.chunks.size() * sizeof(ChunkDesc));
    L.off_cbeg = take(pl.chunk_begin.size() * sizeof(int));
    L.off_tiles = take(pl.tiles.size() * sizeof(TileDesc));
    L.off_cover = take(pl.cover.size() * sizeof(int));
    L.off_pkts = take(pl.pkts.size() * sizeof(PacketDesc));
    L.host_bytes = o;
    const int tt = std::max(gram_tiles(pl.ntp, false), gram_tiles(pl.ntp, true));
    L.off_wtab = take(pl.wtab_len * sizeof(double));
    L.off_partial = take(pl.chunks.size() * (size_t)tt * 256 * sizeof(float));
    L.off_rwin = take(S * ntp * ntp * sizeof(float2));
    L.off_rext = take(S * nte * nte * sizeof(double2));
    L.off_hv = take(S * RMAX * ntp * sizeof(double2));
    L.off_htau = take(S * RMAX * sizeof(double));
    L.off_vr64 = take(S * ntp * RMAX * sizeof(double2));
    L.off_vr32 = take(S * ntp * RMAX * sizeof(float2));
    L.off_rank = take(S * sizeof(int));
    L.off_bmat = take(S * ntp * ntp * sizeof(double2));
    L.off_wvec = take(S * ntp * ntp * sizeof(double2));
    L.off_lam = take(S * ntp * sizeof(double));
    L.off_wts = take(S * ntp * sizeof(double));
    L.off_kcut = take(S * sizeof(int));
    L.off_flags = take(S * sizeof(int));
    L.off_sweeps = take(S * sizeof(int));
    L.off_alpha = take(S * sizeof(double));
    L.off_curve = take(S * ntp * sizeof(double));
    L.off_pmat = take(S * ntp * ntp * sizeof(double2));
    L.off_breal = take(S * (2 * nte) * (2 * ntp) * sizeof(float));
    L.total = o;
    return L;
}

Workspace make_ws(char* base, const Layout& L, const Plan& pl, const float* explicit_w) {
    Workspace ws;
    ws.S = (int)pl.sub.size();
    ws.ntp = pl.ntp;
    ws.nte = pl.ntp + REXT;
    ws.sub = (const SubsetDesc*)(base + L.off_sub);
    ws.chunks = (const ChunkDesc*)(base + L.off_chunks);
    ws.nchunks = (int)pl.chunks.size();
    ws.chunk_begin = (const int*)(base + L.off_cbeg);
    ws.tiles = (const TileDesc*)(base + L.off_tiles);
    ws.ntiles = (int)pl.tiles.size();
    ws.trows = pl.trows;
    ws.rvar = pl.rvar;
    ws.cover = (const int*)(base + L.off_cover);
    ws.pkts = (const PacketDesc*)(base + L.off_pkts);
    ws.wtab = (double*)(base + L.off_wtab);
    ws.partial = (float*)(base + L.off_partial);
    ws.rwin = (float2*)(base + L.off_rwin);
    ws.rext = (double2*)(base + L.off_rext);
    ws.hv = (double2*)(base + L.off_hv);
    ws.htau = (double*)(base + L.off_htau);
    ws.vr64 = (double2*)(base + L.off_vr64);
    ws.vr32 = (float2*)(base + L.off_vr32);
    ws.rank = (int*)(base + L.off_rank);
    ws.bmat = (double2*)(base + L.off_bmat);
    ws.wvec = (double2*)(base + L.off_wvec);
    ws.lam = (double*)(base + L.off_lam);
    ws.wts = (double*)(base + L.off_wts);
    ws.kcut = (int*)(base + L.off_kcut);
    ws.flags = (int*)(base + L.off_flags);
    ws.sweeps = (int*)(base + L.off_sweeps);
    ws.alpha = (double*)(base + L.off_alpha);
    ws.curve = (double*)(base + L.off_curve);
    ws.pmat = (double2*)(base + L.off_pmat);
    ws.breal = (float*)(base + L.off_breal);
    ws.explicit_w = explicit_w;
    return ws;
}

// A view of the workspace restricted to subset s (sequential schedule). The
// chunk table of the view lives at `chunks` with subset index 0.
Workspace subset_view(const Workspace& w, int s, const ChunkDesc* chunks, const int* cbeg, int nch) {
    Workspace v = w;
    const long ntp = w.ntp, nte = w.nte;
    v.S = 1;
    v.sub = w.sub + s;
    v.chunks = chunks;
    v.nchunks = nch;
    v.chunk_begin = cbeg;
    v.rwin = w.rwin + s * ntp * ntp;
    v.rext = w.rext + s * nte * nte;
    v.hv = w.hv + s * RMAX * ntp;
    v.htau = w.htau + s * RMAX;
    v.vr64 = w.vr64 + s * ntp * RMAX;
    v.vr32 = w.vr32 + s * ntp * RMAX;
    v.rank = w.rank + s;
    v.bmat = w.bmat + s * ntp * ntp;
    v.wvec = w.wvec + s * ntp * ntp;
    v.lam = w.lam + s * ntp;
    v.wts = w.wts + s * ntp;
    v.kcut = w.kcut + s;
    v.flags = w.flags + s;
    v.sweeps = w.sweeps + s;
    v.alpha = w.alpha + s;
    v.curve = w.curve + s * ntp;
    v.pmat = w.pmat + s * ntp * ntp;
    v.breal = w.breal + s * (2 * nte) * (2 * ntp);
    return v;
}

#define HIPCHK(x)                                        \
    do {                                                 \
        if ((x) != hipSuccess) return LCF_ERR_DEVICE;    \
    } while (0)

// Resolve recorded event pairs into the per-stage totals.
hipError_t drain_timing(lcf_context* c) {
    for (auto& pe : c->evpending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(c->evpool[pe.second + 1]);
        if (e != hipSuccess) return e;
        e = hipEventElapsedTime(&ms, c->evpool[pe.second], c->evpool[pe.second + 1]);
        if (e != hipSuccess) return e;
        c->stage_ms[pe.first] += ms;
        c->stage_n[pe.first] += 1;
    }
    c->evpending.clear();
    c->evnext = 0;
    return hipSuccess;
}

// Bracket one launch with events when timing is on: tick() before, tock() after.
struct StageScope {
    lcf_context* c;
    int stage;
    hipStream_t st;
    size_t idx = 0;
    bool on = false;
    StageScope(lcf_context* c_, int stage_, hipStream_t st_) : c(c_), stage(stage_), st(st_) {
        if (!c->timing) return;
        if (c->evnext + 2 > c->evpool.size()) {
            // events already recorded are resolved first; if that fails, this stage is not timed
            if (c->evnext + 2 > 4096 && drain_timing(c) != hipSuccess) return;
            while (c->evnext + 2 > c->evpool.size()) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                c->evpool.push_back(e);
            }
        }
        idx = c->evnext;
        c->evnext += 2;
        on = hipEventRecord(c->evpool[idx], st) == hipSuccess;
    }
    ~StageScope() {
        if (!on) return;
        if (hipEventRecord(c->evpool[idx + 1], st) == hipSuccess) c->evpending.push_back({stage, idx});
    }
};
#define STAGE(c, s, st) StageScope _scope_##s(c, s, st)

// Covariance passes, tissue basis and assembly. `cov` (may be null) receives R
// of the `nsub` subsets of this view in the original basis (diagnostics).
lcf_status run_stages(lcf_context* c, const Workspace& ws, const lcf_threshold* thr, int prec,
                      double2* cov, int nt, hipStream_t st) {
    { STAGE(c, LCF_STAGE_WINDOWS, st); HIPCHK(launch_windows(ws, st)); }
    { STAGE(c, LCF_STAGE_GRAM1, st); HIPCHK(launch_gram(ws, false, false, prec, st)); }
    { STAGE(c, LCF_STAGE_GRAM1_REDUCE, st); HIPCHK(launch_gram(ws, false, true, prec, st)); }
    { STAGE(c, LCF_STAGE_TISSUE, st); HIPCHK(launch_tissue(ws, thr->deflate_rho, c->sub_iters, st)); }
    { STAGE(c, LCF_STAGE_GRAM2, st); HIPCHK(launch_gram(ws, true, false, prec, st)); }
    { STAGE(c, LCF_STAGE_GRAM2_REDUCE, st); HIPCHK(launch_gram(ws, true, true, prec, st)); }
    { STAGE(c, LCF_STAGE_ASSEMBLE, st); HIPCHK(launch_assemble(ws, cov != nullptr, st)); }
    if (cov) HIPCHK(launch_export_cov(ws, 0, ws.S, nt, cov, st));
    return LCF_OK;
}

lcf_status run_stages2(lcf_context* c, const Workspace& ws, const lcf_threshold* thr, int prec, int nt_max,
                       int all_vectors, float* mlp_scratch, int evd, hipStream_t st) {
    const bool mlp = thr->cut == LCF_CUT_MLP;
    RuleParams rp{mlp ? (int)LCF_CUT_KNEE : thr->cut, thr->shape, thr->pd_mode, thr->k_fixed, thr->beta_knee,
                  thr->knee_max_frac, thr->beta_sigmoid, thr->beta_median, thr->slope_thr, thr->beta_power};
    { STAGE(c, LCF_STAGE_EVD, st); HIPCHK(launch_evd(ws, c->max_sweeps, nt_max, evd, st)); }
    const bool ncc = thr->cut == LCF_CUT_NCC;
    if (ncc) {
        // method 4 reads every eigenvector before the cut is known
        { STAGE(c, LCF_STAGE_EVD_VECTORS, st); HIPCHK(launch_evd_vectors(ws, evd, 1, c->max_sweeps, nt_max, st)); }
        { STAGE(c, LCF_STAGE_NCC, st); HIPCHK(launch_ncc(ws, st)); }
    }
    { STAGE(c, LCF_STAGE_RULES, st); HIPCHK(launch_rules(ws, rp, st)); }
    if (mlp) {
        STAGE(c, LCF_STAGE_MLP, st);
        // scratch laid out as [valid ints][z | h1 a1 h2 a2 | w]; sized by the caller
        int* valid = (int*)mlp_scratch;
        float* z = mlp_scratch + align_up((size_t)ws.S, 64);
        float* act = z + (size_t)ws.S * MLP_NT;
        float* wout = act + (size_t)ws.S * 4 * MLP_H;
        if (ws.ntp == MLP_NT) {
            HIPCHK(mlp_features(ws.lam, ws.ntp, ws.S, z, valid, st));
            HIPCHK(mlp_forward(c->mlp, z, ws.S, act, wout, st));
            HIPCHK(mlp_apply(ws, wout, valid, thr->pd_mode, c->mlp_gate_mdb < 0 ? -1.0 : 1e-3 * c->mlp_gate_mdb,
                             ws.curve, st));
        } else {
            HIPCHK(mlp_apply(ws, wout, nullptr, thr->pd_mode, -1.0, ws.curve, st));   // all subsets keep the rule
        }
    }
    if (!ncc) {
        STAGE(c, LCF_STAGE_EVD_VECTORS, st);
        HIPCHK(launch_evd_vectors(ws, evd, all_vectors, c->max_sweeps, nt_max, st));
    }
    { STAGE(c, LCF_STAGE_PROJECTOR, st); HIPCHK(launch_projector(ws, prec, st)); }
    return LCF_OK;
}

// A launch group staged on the device: plan descriptors uploaded, workspace
// views set up.
struct Staged {
    Workspace ws;
    char* base = nullptr;          // device block holding descriptors and workspace
    size_t seq_off = 0;
    float* mlp_scratch = nullptr;  // network activations (learned weights only)
};

// A fixed device block that a call must fit in (the allocation-free entry
// point): nothing is grown, plans that do not fit are refused.
struct FixedArena {
    char* base;
    size_t cap;
};

lcf_status stage_group(lcf_context* c, const Plan& pl, const lcf_threshold* thr, hipStream_t st, Staged& sg,
                       const FixedArena* fx = nullptr) {
    Layout L = make_layout(pl);
    // sequential schedule: per-subset chunk tables appended to the host block
    const size_t seq_off = L.host_bytes;
    size_t seq_bytes = 0;
    if (c->schedule == 1) seq_bytes = pl.chunks.size() * sizeof(ChunkDesc) + 2 * pl.sub.size() * sizeof(int);
    const size_t host_total = align_up(L.host_bytes + seq_bytes, 256);
    // shift device-only buffers after the host block
    Layout D = L;
    const size_t shift = host_total - L.host_bytes;
    for (size_t* p = &D.off_wtab; p <= &D.off_breal; ++p) *p += shift;
    D.total += shift;
    const size_t mlp_floats = thr->cut == LCF_CUT_MLP
                                  ? align_up(pl.sub.size(), 64) + mlp_infer_scratch_floats((int)pl.sub.size())
                                  : 0;
    char* h = nullptr;
    char* base = nullptr;
    if (fx) {
        // everything, network activations included, inside the caller-visible fixed block
        if (D.total + mlp_floats * sizeof(float) > fx->cap) return LCF_ERR_SCRATCH_LIMIT;
        if (c->fixed_pending) {
            if (hipEventSynchronize(c->fixed_staged) != hipSuccess) return LCF_ERR_DEVICE;
            c->fixed_pending = false;
        }
        if (c->fixed_host.size() < host_total) c->fixed_host.resize(host_total);
        h = c->fixed_host.data();
        base = fx->base;
    } else {
        lcf_status e = ensure_device(c, D.total);
        if (e != LCF_OK) return e;
        e = ensure_host(c, host_total);
        if (e != LCF_OK) return e;
        h = c->hbuf;
        base = c->dbuf;
    }
    std::memcpy(h + L.off_sub, pl.sub.data(), pl.sub.size() * sizeof(SubsetDesc));
    std::memcpy(h + L.off_chunks, pl.chunks.data(), pl.chunks.size() * sizeof(ChunkDesc));
    std::memcpy(h + L.off_cbeg, pl.chunk_begin.data(), pl.chunk_begin.size() * sizeof(int));
    std::memcpy(h + L.off_tiles, pl.tiles.data(), pl.tiles.size() * sizeof(TileDesc));
    std::memcpy(h + L.off_cover, pl.cover.data(), pl.cover.size() * sizeof(int));
    std::memcpy(h + L.off_pkts, pl.pkts.data(), pl.pkts.size() * sizeof(PacketDesc));
    if (c->schedule == 1) {
        ChunkDesc* sc = (ChunkDesc*)(h + seq_off);
        for (size_t i = 0; i < pl.chunks.size(); ++i) { sc[i] = pl.chunks[i]; sc[i].s = 0; }
        int* cb = (int*)(h + seq_off + pl.chunks.size() * sizeof(ChunkDesc));
        for (size_t s = 0; s < pl.sub.size(); ++s) {
            cb[2 * s] = 0;
            cb[2 * s + 1] = pl.chunk_begin[s + 1] - pl.chunk_begin[s];
        }
    }
    HIPCHK(hipMemcpyAsync(base, h, host_total, hipMemcpyHostToDevice, st));
    if (fx) {
        HIPCHK(hipEventRecord(c->fixed_staged, st));
        c->fixed_pending = true;
    } else {
        HIPCHK(hipEventRecord(c->staged, st));
        c->staged_pending = true;
    }
    sg.ws = make_ws(base, D, pl, thr->cut == LCF_CUT_EXPLICIT ? thr->explicit_w : nullptr);
    sg.base = base;
    sg.seq_off = seq_off;
    if (thr->cut == LCF_CUT_MLP) {
        if (fx) {
            sg.mlp_scratch = (float*)(base + D.total);
        } else {
            lcf_status e = ensure_mlp_scratch(c, mlp_floats);
            if (e != LCF_OK) return e;
            sg.mlp_scratch = c->mlp_scratch;
        }
    }
    return LCF_OK;
}

// The launch chain of one staged group (every stage through the reprojection).
lcf_status run_chain(lcf_context* c, const Plan& pl, const Staged& sg, const lcf_threshold* thr, int prec,
                     const lcf_diag* diag, hipStream_t st) {
    const Workspace& ws = sg.ws;
    const int evd = pl.evd >= 0 ? pl.evd : c->evd_method;
    lcf_status e;
    if (c->schedule == 1) {
        // the paper's loop: one subset at a time through every per-subset stage
        const ChunkDesc* dch = (const ChunkDesc*)(sg.base + sg.seq_off);
        const int* dcb = (const int*)(sg.base + sg.seq_off + pl.chunks.size() * sizeof(ChunkDesc));
        for (int s = 0; s < (int)pl.sub.size(); ++s) {
            const int cb0 = pl.chunk_begin[s], nch = pl.chunk_begin[s + 1] - cb0;
            Workspace v = subset_view(ws, s, dch + cb0, dcb + 2 * s, nch);
            double2* cv = (diag && diag->cov) ? (double2*)diag->cov + (long)s * pl.sub[s].nt * pl.sub[s].nt : nullptr;
            e = run_stages(c, v, thr, prec, cv, pl.sub[s].nt, st);
            if (e != LCF_OK) return e;
            e = run_stages2(c, v, thr, prec, pl.sub[s].nt, diag && diag->eigvecs ? 1 : 0, sg.mlp_scratch, evd, st);
            if (e != LCF_OK) return e;
        }
    } else {
        e = run_stages(c, ws, thr, prec, diag ? (double2*)diag->cov : nullptr, pl.sub[0].nt, st);
        if (e != LCF_OK) return e;
        e = run_stages2(c, ws, thr, prec, pl.nt_max, diag && diag->eigvecs ? 1 : 0, sg.mlp_scratch, evd, st);
        if (e != LCF_OK) return e;
    }
    { STAGE(c, LCF_STAGE_REPROJ, st); HIPCHK(launch_reproj(ws, prec, st)); }
    if (diag)
        HIPCHK(launch_export(ws, 0, (int)pl.sub.size(), pl.sub[0].nt, diag->eigvals, diag->weights, diag->k,
                             diag->sweeps, diag->flags, diag->alpha, diag->rank, (double2*)diag->eigvecs,
                             thr->cut == LCF_CUT_NCC ? diag->curve : nullptr,
                             thr->cut == LCF_CUT_MLP ? diag->mlp_gate : nullptr, st));
    HIPCHK(launch_flags_or(ws, c->sticky, st));
    return LCF_OK;
}

// Autotuner key of a launch group: padded Nt class, precision, schedule and
// the log2 classes of the subset count and of the mean box size.
std::string tune_key(const Plan& pl, int prec, int schedule) {
    double neff = 0.0;
    for (const SubsetDesc& sd : pl.sub) neff += sd.neff;
    neff /= std::max<size_t>(1, pl.sub.size());
    const int sc = (int)std::floor(std::log2((double)std::max<size_t>(1, pl.sub.size())));
    const int nc = (int)std::floor(std::log2(std::max(1.0, neff)));
    char buf[96];
    std::snprintf(buf, sizeof buf, "ntp%d_p%d_s%d_S%d_N%d", pl.ntp, prec, schedule, sc, nc);
    return buf;
}

// Time every (split-K chunk, reprojection tile) candidate on the caller's
// packets with HIP events (one untimed run, one timed run each) and keep the
// fastest; then, up to 128 frames, the other subset EVD method (tridiagonal
// solver or Jacobi) on the winning plan. The outputs end up written by the last
// candidate; the caller's run overwrites them.
lcf_status tune_group(lcf_context* c, const std::vector<PacketIn>& in, const std::vector<int>& idx,
                      const lcf_threshold* thr, int prec, hipStream_t st, const std::string& key) {
    static const int chunks[] = {512, 1024, 2048, 4096};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return LCF_ERR_DEVICE; }
    const int saved_timing = c->timing;
    c->timing = 0;
    float best = 0.f;
    TuneChoice choice{CHUNK, 2, 0, c->evd_method};
    lcf_status res = LCF_OK;
    int ntp = 0;
    for (int i : idx) ntp = std::max(ntp, ntp_class(in[i].g.nt));
    auto trial = [&](int ch, int rows, int var, int evd) -> bool {
        Plan pl;
        build_plan(pl, in, idx, thr->pd_mode, ch, rows, var);
        pl.evd = evd;
        Staged sg;
        res = stage_group(c, pl, thr, st, sg);
        if (res != LCF_OK) return false;
        res = run_chain(c, pl, sg, thr, prec, nullptr, st);
        if (res != LCF_OK) return false;
        if (hipEventRecord(e0, st) != hipSuccess) { res = LCF_ERR_DEVICE; return false; }
        res = run_chain(c, pl, sg, thr, prec, nullptr, st);
        if (res != LCF_OK) return false;
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { res = LCF_ERR_DEVICE; return false; }
        if (best == 0.f || ms < best) { best = ms; choice = TuneChoice{ch, rows, var, evd}; }
        return true;
    };
    std::vector<std::pair<int, int>> tiles = {{2, 0}};                 // (rows, variant)
    if (trows_max(ntp) >= 4) {
        tiles.push_back({4, 0});
        if (prec == LCF_PREC_FP32) tiles.push_back({4, 1});       // producer/consumer: FP32 only
    }
    for (const auto& tv : tiles)
        for (int ch : chunks)
            if (!trial(ch, tv.first, tv.second, c->evd_method)) goto done;
    if (ntp <= 128) trial(choice.chunk, choice.trows, choice.rvar, 1 - c->evd_method);
done:
    c->timing = saved_timing;
    (void)hipEventDestroy(e0);     // the trial timings are already read
    (void)hipEventDestroy(e1);
    if (res == LCF_OK) c->tuned[key] = choice;
    return res;
}

// Filter a list of packets. diag applies to a single packet call only.
lcf_status filter_packets(lcf_context* c, const std::vector<PacketIn>& in, const lcf_threshold* thr, int prec,
                          const lcf_diag* diag, hipStream_t st, const FixedArena* fx = nullptr) {
    if (!c) return LCF_ERR_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return LCF_ERR_DEVICE;
    // A call made while the caller captures the stream is refused: the plan
    // upload and the workspace of a captured chain would be overwritten or
    // reallocated by later calls before the caller's graph is replayed.
    lcf_status ce = refuse_capture(st);
    if (ce != LCF_OK) return ce;
    // group packets by padded Nt class
    std::map<int, std::vector<int>> groups;
    for (size_t i = 0; i < in.size(); ++i) groups[ntp_class(in[i].g.nt)].push_back((int)i);
    for (auto& kv : groups) {
        // plan parameters: the tuned choice for this group's class, else the defaults
        Plan pl;
        // default: 4-row tiles where allowed; producer/consumer waves for the FP32
        // GEMM (measured faster there), one role per wave for split BF16
        build_plan(pl, in, kv.second, thr->pd_mode, CHUNK, trows_max(kv.first),
                   (trows_max(kv.first) >= 4 && prec == LCF_PREC_FP32) ? 1 : 0);
        const std::string tkey = tune_key(pl, prec, c->schedule);
        auto tit = c->tuned.find(tkey);
        if (tit == c->tuned.end() && c->autotune && !fx) {
            lcf_status e = tune_group(c, in, kv.second, thr, prec, st, tkey);
            if (e != LCF_OK) return e;
            tit = c->tuned.find(tkey);
        }
        if (tit != c->tuned.end()) {
            const int tr = std::min(tit->second.trows, trows_max(kv.first));
            const int rv = tr == 4 ? tit->second.rvar : 0;
            if (tit->second.chunk != pl.chunk || tr != pl.trows || rv != pl.rvar) {
                Plan tuned;
                build_plan(tuned, in, kv.second, thr->pd_mode, tit->second.chunk, tr, rv);
                pl = std::move(tuned);
            }
            pl.evd = kv.first <= 128 ? tit->second.evd : -1;
        }
        Staged sg;
        lcf_status e = stage_group(c, pl, thr, st, sg, fx);
        if (e != LCF_OK) return e;
        // Launch chain of the group, optionally captured once into a hipGraph and
        // replayed for later calls with the same plan (not on the null stream, not
        // while stage timing is on, and not for the fixed block, whose chains are
        // launched directly).
        const bool graph = c->use_graph && !c->timing && st != nullptr && !fx;
        std::string key;
        if (graph) {
            key = graph_key(c, pl, in, kv.second, thr, prec, diag);
            auto it = c->graphs.find(key);
            if (it != c->graphs.end()) {
                HIPCHK(hipGraphLaunch(it->second, st));
                continue;
            }
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        }
        e = run_chain(c, pl, sg, thr, prec, diag, st);
        if (graph) {
            hipGraph_t gr = nullptr;
            const hipError_t ce = hipStreamEndCapture(st, &gr);
            if (e != LCF_OK) { if (gr) (void)hipGraphDestroy(gr); return e; }
            if (ce != hipSuccess) return LCF_ERR_DEVICE;
            hipGraphExec_t ex = nullptr;
            const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);     // the executable graph does not need it
            if (ie != hipSuccess) return LCF_ERR_DEVICE;
            c->graphs[key] = ex;
            HIPCHK(hipGraphLaunch(ex, st));
        } else if (e != LCF_OK) {
            return e;
        }
    }
    return LCF_OK;
}

// One push of a sliding-packet stream: the covariance from the previous
// packet's by the hop, then every stage after the Gram passes.
lcf_status stream_chain(lcf_context* c, const Plan& pl, const Staged& sg, const lcf_threshold* thr, int prec,
                        const double2* rold, double2* rnew, double2* part, int hop, const lcf_diag* diag,
                        hipStream_t st) {
    const Workspace& ws = sg.ws;
    { STAGE(c, LCF_STAGE_WINDOWS, st); HIPCHK(launch_windows(ws, st)); }
    { STAGE(c, LCF_STAGE_COV_STREAM, st); HIPCHK(launch_cov_stream(ws, rold, rnew, part, hop, st)); }
    { STAGE(c, LCF_STAGE_TISSUE, st); HIPCHK(launch_tissue(ws, thr->deflate_rho, c->sub_iters, st)); }
    const bool cov = diag && diag->cov;
    { STAGE(c, LCF_STAGE_ASSEMBLE, st); HIPCHK(launch_assemble(ws, cov, st)); }
    if (cov) HIPCHK(launch_export_cov(ws, 0, ws.S, pl.sub[0].nt, (double2*)diag->cov, st));
    lcf_status e = run_stages2(c, ws, thr, prec, pl.nt_max, diag && diag->eigvecs ? 1 : 0, sg.mlp_scratch,
                               c->evd_method, st);
    if (e != LCF_OK) return e;
    { STAGE(c, LCF_STAGE_REPROJ, st); HIPCHK(launch_reproj(ws, prec, st)); }
    if (diag)
        HIPCHK(launch_export(ws, 0, (int)pl.sub.size(), pl.sub[0].nt, diag->eigvals, diag->weights, diag->k,
                             diag->sweeps, diag->flags, diag->alpha, diag->rank, (double2*)diag->eigvecs,
                             thr->cut == LCF_CUT_NCC ? diag->curve : nullptr,
                             thr->cut == LCF_CUT_MLP ? diag->mlp_gate : nullptr, st));
    HIPCHK(launch_flags_or(ws, c->sticky, st));
    return LCF_OK;
}

}  // namespace

extern "C" {

lcf_status lcf_create(int32_t device, lcf_context** out) {
    if (!out) return LCF_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LCF_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_context* c = new lcf_context();
    c->device = device;
    if (init_scratch_ptr(device) != LCF_OK) {
        delete c;
        return LCF_ERR_DEVICE;
    }
    if (hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fixed_staged, hipEventDisableTiming) != hipSuccess ||
        hipMalloc((void**)&c->sticky, sizeof(int)) != hipSuccess ||
        hipMemset(c->sticky, 0, sizeof(int)) != hipSuccess) {
        delete c;
        return LCF_ERR_DEVICE;
    }
    *out = c;
    return LCF_OK;
}

lcf_status lcf_destroy(lcf_context* c) {
    if (!c) return LCF_OK;
    // everything is released even after a failure; the first error is reported
    hipError_t first = hipSuccess;
    auto note = [&](hipError_t e) { if (first == hipSuccess && e != hipSuccess) first = e; };
    note(hipSetDevice(c->device));
    note(hipDeviceSynchronize());
    for (auto& kv : c->graphs) note(hipGraphExecDestroy(kv.second));
    for (auto e : c->evpool) note(hipEventDestroy(e));
    for (void* p : {(void*)c->mlp.master, (void*)c->mlp.wbf, (void*)c->mlp.m, (void*)c->mlp.v, (void*)c->mlp.grad,
                    (void*)c->mlp_scratch})
        if (p) note(hipFree(p));
    if (c->dbuf) note(hipFree(c->dbuf));
    if (c->hbuf) note(hipHostFree(c->hbuf));
    if (c->sticky) note(hipFree(c->sticky));
    if (c->staged) note(hipEventDestroy(c->staged));
    if (c->fixed_staged) note(hipEventDestroy(c->fixed_staged));
    delete c;
    return first == hipSuccess ? LCF_OK : LCF_ERR_DEVICE;
}

lcf_status lcf_set_option(lcf_context* c, int32_t option, int64_t value) {
    if (!c) return LCF_ERR_INVALID_ARG;
    switch (option) {
        case LCF_OPT_SCHEDULE:
            if (value != 0 && value != 1) return LCF_ERR_INVALID_ARG;
            c->schedule = (int)value;
            return LCF_OK;
        case LCF_OPT_MAX_SWEEPS:
            if (value < 1 || value > 1000) return LCF_ERR_INVALID_ARG;
            c->max_sweeps = (int)value;
            return LCF_OK;
        case LCF_OPT_USE_GRAPH:
            if (value != 0 && value != 1) return LCF_ERR_INVALID_ARG;
            c->use_graph = (int)value;
            return LCF_OK;
        case LCF_OPT_SUBSPACE_IT:
            if (value < 1 || value > 100) return LCF_ERR_INVALID_ARG;
            c->sub_iters = (int)value;
            return LCF_OK;
        case LCF_OPT_STAGE_TIMING:
            if (value != 0 && value != 1) return LCF_ERR_INVALID_ARG;
            c->timing = (int)value;
            return LCF_OK;
        case LCF_OPT_AUTOTUNE:
            if (value != 0 && value != 1) return LCF_ERR_INVALID_ARG;
            c->autotune = (int)value;
            return LCF_OK;
        case LCF_OPT_MLP_GATE:
            if (value < -1 || value > 1000000) return LCF_ERR_INVALID_ARG;
            c->mlp_gate_mdb = (long)value;
            return LCF_OK;
        case LCF_OPT_EVD:
            if (value != 0 && value != 1) return LCF_ERR_INVALID_ARG;
            c->evd_method = (int)value;
            drop_graphs(c);
            return LCF_OK;
        default:
            return LCF_ERR_INVALID_ARG;
    }
}

lcf_status lcf_validate(const lcf_geometry* geo, const lcf_threshold* thr, int32_t precision) {
    lcf_status e = validate_geometry(geo);
    if (e != LCF_OK) return e;
    e = validate_threshold(thr, geo->nt);
    if (e != LCF_OK) return e;
    return validate_precision(precision);
}

lcf_status lcf_filter(lcf_context* ctx, const lcf_geometry* geo, const lcf_threshold* thr, int32_t precision,
                      const void* iq, void* iq_out, float* pd, const lcf_diag* diag, void* stream) {
    if (!ctx || !iq || !pd) return LCF_ERR_INVALID_ARG;
    lcf_status e = lcf_validate(geo, thr, precision);
    if (e != LCF_OK) return e;
    if (thr->cut == LCF_CUT_MLP && !ctx->mlp_ready) return LCF_ERR_MODEL;
    std::vector<PacketIn> in{PacketIn{*geo, iq, iq_out, pd, 0}};
    return filter_packets(ctx, in, thr, precision, diag, (hipStream_t)stream);
}

lcf_status lcf_filter_noalloc(lcf_context* ctx, const lcf_geometry* geo, const lcf_threshold* thr,
                              int32_t precision, const void* iq, void* iq_out, float* pd, const lcf_diag* diag,
                              void* stream) {
    if (!ctx || !iq || !pd) return LCF_ERR_INVALID_ARG;
    lcf_status e = lcf_validate(geo, thr, precision);
    if (e != LCF_OK) return e;
    if (thr->cut == LCF_CUT_MLP && !ctx->mlp_ready) return LCF_ERR_MODEL;
    char* base = scratch_ptr(ctx->device);
    if (!base) return LCF_ERR_DEVICE;
    const FixedArena fx{base, (size_t)LCF_NOALLOC_SCRATCH_BYTES};
    std::vector<PacketIn> in{PacketIn{*geo, iq, iq_out, pd, 0}};
    return filter_packets(ctx, in, thr, precision, diag, (hipStream_t)stream, &fx);
}

lcf_status lcf_filter_batch(lcf_context* ctx, int32_t n, const lcf_geometry* geo, const lcf_threshold* thr,
                            int32_t precision, const void* const* iq, void* const* iq_out, float* const* pd,
                            void* stream) {
    if (!ctx || n < 1 || !geo || !iq || !pd || !thr) return LCF_ERR_INVALID_ARG;
    std::vector<PacketIn> in;
    long ew = 0;     // caller-given weights: packets' [nd][nt] blocks back to back
    for (int i = 0; i < n; ++i) {
        lcf_status e = lcf_validate(&geo[i], thr, precision);
        if (e != LCF_OK) return e;
        if (!iq[i] || !pd[i]) return LCF_ERR_INVALID_ARG;
        if (thr->cut == LCF_CUT_MLP && !ctx->mlp_ready) return LCF_ERR_MODEL;
        in.push_back(PacketIn{geo[i], iq[i], iq_out ? iq_out[i] : nullptr, pd[i], ew});
        ew += (long)geo[i].gy * geo[i].gx * geo[i].nt;
    }
    return filter_packets(ctx, in, thr, precision, nullptr, (hipStream_t)stream);
}

lcf_status lcf_stream_create(lcf_context* ctx, const lcf_geometry* geo, const lcf_threshold* thr,
                             int32_t precision, lcf_stream** out) {
    if (!ctx || !out) return LCF_ERR_INVALID_ARG;
    *out = nullptr;
    lcf_status e = lcf_validate(geo, thr, precision);
    if (e != LCF_OK) return e;
    if (thr->cut == LCF_CUT_MLP && !ctx->mlp_ready) return LCF_ERR_MODEL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_stream* sm = new lcf_stream();
    sm->ctx = ctx;
    sm->geo = *geo;
    sm->thr = *thr;
    sm->prec = precision;
    const int ntp = ntp_class(geo->nt);
    std::vector<PacketIn> in{PacketIn{*geo, nullptr, nullptr, nullptr, 0}};
    build_plan(sm->plan, in, std::vector<int>{0}, thr->pd_mode, CHUNK, trows_max(ntp),
               (trows_max(ntp) >= 4 && precision == LCF_PREC_FP32) ? 1 : 0);
    const size_t S = sm->plan.sub.size();
    const size_t rbytes = S * ntp * ntp * sizeof(double2);
    const size_t pbytes = stream_partial_elems((int)S, ntp) * sizeof(double2);
    if (hipMalloc((void**)&sm->rbuf[0], rbytes) != hipSuccess || hipMalloc((void**)&sm->rbuf[1], rbytes) != hipSuccess ||
        hipMalloc((void**)&sm->part, pbytes) != hipSuccess) {
        lcf_stream_destroy(sm);
        return LCF_ERR_OUT_OF_MEMORY;
    }
    if (hipMemset(sm->rbuf[0], 0, rbytes) != hipSuccess || hipMemset(sm->rbuf[1], 0, rbytes) != hipSuccess) {
        lcf_stream_destroy(sm);
        return LCF_ERR_DEVICE;
    }
    *out = sm;
    return LCF_OK;
}

lcf_status lcf_stream_push(lcf_stream* sm, const void* iq, int32_t hop, void* iq_out, float* pd,
                           const lcf_diag* diag, void* stream) {
    if (!sm || !iq || !pd) return LCF_ERR_INVALID_ARG;
    const int nt = sm->geo.nt;
    if (hop < 1 || hop > nt) return LCF_ERR_INVALID_ARG;
    lcf_context* c = sm->ctx;
    if (hipSetDevice(c->device) != hipSuccess) return LCF_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    lcf_status e = refuse_capture(st);
    if (e != LCF_OK) return e;
    if (!sm->primed) hop = nt;
    Plan& pl = sm->plan;
    for (SubsetDesc& sd : pl.sub) sd.iq = (const float2*)iq;
    pl.pkts[0].iq = (const float2*)iq;
    pl.pkts[0].iq_out = (float*)iq_out;
    pl.pkts[0].pd = pd;
    Staged sg;
    e = stage_group(c, pl, &sm->thr, st, sg);
    if (e != LCF_OK) return e;
    const int nxt = 1 - sm->cur;
    e = stream_chain(c, pl, sg, &sm->thr, sm->prec, sm->rbuf[sm->cur], sm->rbuf[nxt], sm->part, hop, diag, st);
    if (e != LCF_OK) return e;
    sm->cur = nxt;
    sm->primed = true;
    return LCF_OK;
}

lcf_status lcf_stream_destroy(lcf_stream* sm) {
    if (!sm) return LCF_OK;
    // everything is released even after a failure; the first error is reported
    hipError_t first = hipSuccess;
    auto note = [&](hipError_t e) { if (first == hipSuccess && e != hipSuccess) first = e; };
    note(hipSetDevice(sm->ctx->device));
    note(hipDeviceSynchronize());
    for (void* p : {(void*)sm->rbuf[0], (void*)sm->rbuf[1], (void*)sm->part})
        if (p) note(hipFree(p));
    delete sm;
    return first == hipSuccess ? LCF_OK : LCF_ERR_DEVICE;
}

lcf_status lcf_heevd_batched(lcf_context* ctx, int32_t n, int32_t nt, const double* a, double* w, double* v,
                             int32_t* sweeps, void* stream) {
    if (!ctx || n < 1 || nt < 2 || nt > 256 || !a || !w) return LCF_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_status ce = refuse_capture((hipStream_t)stream);
    if (ce != LCF_OK) return ce;
    const size_t work = align_up((size_t)n * nt * nt * sizeof(double2), 256);
    const size_t extra = align_up((size_t)n * sizeof(int), 256) * 2;
    lcf_status e = ensure_device(ctx, work + extra);
    if (e != LCF_OK) return e;
    double2* wk = (double2*)ctx->dbuf;
    int* sw = sweeps ? sweeps : (int*)(ctx->dbuf + work);
    int* fl = (int*)(ctx->dbuf + work + extra / 2);
    hipStream_t st = (hipStream_t)stream;
    if (hipMemsetAsync(fl, 0, (size_t)n * sizeof(int), st) != hipSuccess) return LCF_ERR_DEVICE;
    if (launch_heevd(n, nt, (const double2*)a, w, (double2*)v, sw, wk, ctx->max_sweeps, fl, st) != hipSuccess)
        return LCF_ERR_DEVICE;
    Workspace fws{};
    fws.S = n;
    fws.flags = fl;
    if (launch_flags_or(fws, ctx->sticky, st) != hipSuccess) return LCF_ERR_DEVICE;
    return LCF_OK;
}

lcf_status lcf_mlp_init(lcf_context* ctx, uint64_t seed) {
    if (!ctx) return LCF_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_status e = ensure_mlp(ctx);
    if (e != LCF_OK) return e;
    std::vector<float> h(MLP_NPARAM, 0.f);
    uint64_t x = seed;
    auto next = [&]() {   // splitmix64 -> uniform [0, 1)
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int rows, int cols) {
        const double bound = std::sqrt(6.0 / cols) * 0.5;
        for (int i = 0; i < rows * cols; ++i) h[off + i] = (float)((2.0 * next() - 1.0) * bound);
    };
    fill(MLP_OFF_W1, MLP_H, MLP_NT);
    fill(MLP_OFF_W2, MLP_H, MLP_H);
    fill(MLP_OFF_W3, MLP_NT, MLP_H);
    for (int i = 0; i < MLP_NT; ++i) h[MLP_OFF_B3 + i] = 2.0f;
    return lcf_mlp_set_params(ctx, h.data(), MLP_NPARAM);
}

lcf_status lcf_mlp_set_params(lcf_context* ctx, const float* host, int64_t n) {
    if (!ctx || !host || n != MLP_NPARAM) return LCF_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_status e = ensure_mlp(ctx);
    if (e != LCF_OK) return e;
    if (hipMemcpy(ctx->mlp.master, host, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(ctx->mlp.m, 0, n * sizeof(float)) != hipSuccess ||
        hipMemset(ctx->mlp.v, 0, n * sizeof(float)) != hipSuccess)
        return LCF_ERR_DEVICE;
    if (mlp_refresh_bf16(ctx->mlp, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return LCF_ERR_DEVICE;
    ctx->mlp_step = 0;
    ctx->mlp_ready = true;
    return LCF_OK;
}

static lcf_status mlp_copy_out(lcf_context* ctx, const float* src, float* host, int64_t n) {
    if (!ctx || !host || n != MLP_NPARAM) return LCF_ERR_INVALID_ARG;
    if (!ctx->mlp_ready) return LCF_ERR_MODEL;
    if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return LCF_ERR_DEVICE;
    if (hipMemcpy(host, src, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return LCF_ERR_DEVICE;
    return LCF_OK;
}

lcf_status lcf_mlp_get_params(lcf_context* ctx, float* host, int64_t n) {
    return mlp_copy_out(ctx, ctx ? ctx->mlp.master : nullptr, host, n);
}

lcf_status lcf_mlp_get_grads(lcf_context* ctx, float* host, int64_t n) {
    return mlp_copy_out(ctx, ctx ? ctx->mlp.grad : nullptr, host, n);
}

namespace {
struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t nparam;
    uint64_t step;
};
}

lcf_status lcf_mlp_save(lcf_context* ctx, const char* path) {
    if (!ctx || !path) return LCF_ERR_INVALID_ARG;
    if (!ctx->mlp_ready) return LCF_ERR_MODEL;
    const size_t n = MLP_NPARAM;
    std::vector<float> buf(3 * n);
    if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(buf.data(), ctx->mlp.master, n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(buf.data() + n, ctx->mlp.m, n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(buf.data() + 2 * n, ctx->mlp.v, n * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return LCF_ERR_DEVICE;
    CkptHeader hd;
    std::memcpy(hd.magic, "LCFMLP01", 8);
    hd.version = 1;
    hd.nparam = (uint32_t)n;
    hd.step = (uint64_t)ctx->mlp_step;
    uint32_t crc = crc32_update(0, &hd, sizeof(hd));
    crc = crc32_update(crc, buf.data(), buf.size() * 4);
    FILE* f = std::fopen(path, "wb");
    if (!f) return LCF_ERR_INVALID_ARG;
    const bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size() &&
                    std::fwrite(&crc, 4, 1, f) == 1;
    std::fclose(f);
    return ok ? LCF_OK : LCF_ERR_INVALID_ARG;
}

lcf_status lcf_mlp_load(lcf_context* ctx, const char* path) {
    if (!ctx || !path) return LCF_ERR_INVALID_ARG;
    const size_t n = MLP_NPARAM;
    FILE* f = std::fopen(path, "rb");
    if (!f) return LCF_ERR_MODEL;
    CkptHeader hd;
    std::vector<float> buf(3 * n);
    uint32_t crc_file = 0;
    const bool ok = std::fread(&hd, sizeof(hd), 1, f) == 1 && std::memcmp(hd.magic, "LCFMLP01", 8) == 0 &&
                    hd.version == 1 && hd.nparam == n && std::fread(buf.data(), 4, buf.size(), f) == buf.size() &&
                    std::fread(&crc_file, 4, 1, f) == 1;
    std::fclose(f);
    if (!ok) return LCF_ERR_MODEL;
    uint32_t crc = crc32_update(0, &hd, sizeof(hd));
    crc = crc32_update(crc, buf.data(), buf.size() * 4);
    if (crc != crc_file) return LCF_ERR_MODEL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_status e = ensure_mlp(ctx);
    if (e != LCF_OK) return e;
    if (hipMemcpy(ctx->mlp.master, buf.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->mlp.m, buf.data() + n, n * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->mlp.v, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice) != hipSuccess)
        return LCF_ERR_DEVICE;
    if (mlp_refresh_bf16(ctx->mlp, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return LCF_ERR_DEVICE;
    ctx->mlp_step = (long long)hd.step;
    ctx->mlp_ready = true;
    return LCF_OK;
}

lcf_status lcf_mlp_infer(lcf_context* ctx, const double* lam, float* w, int32_t b, void* stream) {
    if (!ctx || !lam || !w || b < 1) return LCF_ERR_INVALID_ARG;
    if (!ctx->mlp_ready) return LCF_ERR_MODEL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_status ce = refuse_capture((hipStream_t)stream);
    if (ce != LCF_OK) return ce;
    lcf_status e = ensure_mlp_scratch(ctx, mlp_infer_scratch_floats(b) + align_up((size_t)b, 64));
    if (e != LCF_OK) return e;
    hipStream_t st = (hipStream_t)stream;
    float* z = ctx->mlp_scratch;
    float* act = z + (size_t)b * MLP_NT;
    if (mlp_features(lam, MLP_NT, b, z, nullptr, st) != hipSuccess) return LCF_ERR_DEVICE;
    if (mlp_forward(ctx->mlp, z, b, act, w, st) != hipSuccess) return LCF_ERR_DEVICE;
    return LCF_OK;
}

lcf_status lcf_mlp_train_step(lcf_context* ctx, const double* lam, const float* target, int32_t b, float lr,
                              float* loss_out, void* stream) {
    if (!ctx || !lam || !target || b < 1 || !(lr >= 0.f)) return LCF_ERR_INVALID_ARG;
    if (!ctx->mlp_ready) return LCF_ERR_MODEL;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    lcf_status ce = refuse_capture((hipStream_t)stream);
    if (ce != LCF_OK) return ce;
    lcf_status e = ensure_mlp_scratch(ctx, mlp_train_scratch_floats(b));
    if (e != LCF_OK) return e;
    ctx->mlp_step += 1;
    if (mlp_train_step(ctx->mlp, lam, target, b, lr, (int)ctx->mlp_step, ctx->mlp_scratch, loss_out,
                       (hipStream_t)stream) != hipSuccess)
        return LCF_ERR_DEVICE;
    return LCF_OK;
}

lcf_status lcf_sync(lcf_context* ctx, void* stream) {
    if (!ctx) return LCF_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return LCF_ERR_DEVICE;
    int f = 0;
    if (hipMemcpy(&f, ctx->sticky, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return LCF_ERR_DEVICE;
    if (f) {
        const int zero = 0;
        if (hipMemcpy(ctx->sticky, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return LCF_ERR_DEVICE;
    }
    if (f & LCF_FLAG_NONFINITE) return LCF_ERR_NONFINITE_INPUT;
    if (f & LCF_FLAG_NO_CONVERGE) return LCF_ERR_NO_CONVERGENCE;
    return LCF_OK;
}

lcf_status lcf_stage_time(lcf_context* ctx, int32_t stage, double* ms, int64_t* launches, int32_t reset) {
    if (!ctx || stage < 0 || stage >= LCF_NUM_STAGES) return LCF_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCF_ERR_DEVICE;
    if (drain_timing(ctx) != hipSuccess) return LCF_ERR_DEVICE;
    if (ms) *ms = ctx->stage_ms[stage];
    if (launches) *launches = ctx->stage_n[stage];
    if (reset)
        for (int i = 0; i < LCF_NUM_STAGES; ++i) { ctx->stage_ms[i] = 0.0; ctx->stage_n[i] = 0; }
    return LCF_OK;
}

lcf_status lcf_tune_save(lcf_context* ctx, const char* path) {
    if (!ctx || !path) return LCF_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "w");
    if (!f) return LCF_ERR_INVALID_ARG;
    bool ok = true;
    for (const auto& kv : ctx->tuned)
        ok = ok && std::fprintf(f, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.chunk, kv.second.trows,
                                kv.second.rvar, kv.second.evd) > 0;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? LCF_OK : LCF_ERR_INVALID_ARG;
}

lcf_status lcf_tune_load(lcf_context* ctx, const char* path) {
    if (!ctx || !path) return LCF_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return LCF_ERR_INVALID_ARG;
    std::map<std::string, TuneChoice> got;
    char line[512], key[128], extra[8];
    bool ok = true;
    while (std::fgets(line, sizeof line, f)) {
        int chunk = 0, rows = 0, var = 0, evd = -1;
        const int n = std::sscanf(line, "%127s %d %d %d %d %7s", key, &chunk, &rows, &var, &evd, extra);
        if (n <= 0) continue;                                       // blank line
        // "<class> <chunk> <rows> <variant> [<evd>]"; files without the EVD column keep the context's
        if ((n != 4 && n != 5) || chunk < PIX || chunk > (1 << 20) || (rows != 2 && rows != 4) || var < 0 ||
            var > 1 || (var == 1 && rows != 4) || evd < -1 || evd > 1) { ok = false; break; }
        got[key] = TuneChoice{chunk, rows, var, evd};
    }
    std::fclose(f);
    if (!ok) return LCF_ERR_INVALID_ARG;
    for (const auto& kv : got) ctx->tuned[kv.first] = kv.second;
    drop_graphs(ctx);
    return LCF_OK;
}

const char* lcf_status_str(lcf_status s) {
    switch (s) {
        case LCF_OK: return "ok";
        case LCF_ERR_INVALID_ARG: return "invalid argument";
        case LCF_ERR_UNSUPPORTED: return "unsupported configuration";
        case LCF_ERR_OUT_OF_MEMORY: return "out of device memory";
        case LCF_ERR_DEVICE: return "HIP device error";
        case LCF_ERR_NONFINITE_INPUT: return "non-finite value reached a covariance";
        case LCF_ERR_NO_CONVERGENCE: return "Jacobi eigen-solver hit the sweep cap";
        case LCF_ERR_MODEL: return "MLP weights missing or corrupt";
        case LCF_ERR_SCRATCH_LIMIT: return "workspace of the call exceeds the fixed block of lcf_filter_noalloc";
    }
    return "unknown status";
}

int32_t lcf_abi_version(void) { return LCF_ABI_VERSION; }

}  // extern "C"
