// Host runtime behind the C ABI of include/dope.h: parameter validation, block partition, device workspace,
// stream-ordered launches of one ADMM iteration (block solves, then consensus and multiplier updates), and
// checkpoint / inspection entry points.
#include "../../include/dope.h"
#include "dope_internal.h"
#include "autotune_table.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

using dope::Ctl;
using dope::Geom;

struct dope_ctx {
    dope_params p{};
    Geom g{};
    int solver = 0;            // resolved: 1 max-flow, 2 exhaustive (0 until set_energy)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    Ctl *ctl = nullptr;
    dope::Img himg{};          // host copy of the device image descriptor (kernel argument of one-image launches)
    bool validate_pending = false;   // a setup is enqueued whose validation no control kernel has taken yet
    bool ctl_fresh = false;          // the device loop control is as the setup kernel leaves it (t = 0, limit
                                     // max_iter, halting on convergence, verdict taken by the first k_finalize):
                                     // a solve needs no control setup
    int32_t *btab = nullptr, *u = nullptr, *w = nullptr, *cw = nullptr, *Y = nullptr, *A0 = nullptr, *A1 = nullptr;
    int32_t *stats = nullptr, *chunk_k0 = nullptr;
    int2 *blist = nullptr;
    uint8_t *yhat = nullptr, *yslot = nullptr, *labels = nullptr;
    int64_t *resid = nullptr, *epart = nullptr;
    int2 *axrow = nullptr;             // axis cover rows (consensus of radius-1 stencils)
    unsigned char *gscr = nullptr;   // per-block max-flow state of blocks beyond the LDS
    Ctl *hctl = nullptr;       // pinned host mirror of the control block
    std::vector<int32_t> hbtab, hchunk;
    int64_t nbl = 0;   // boundary list entries
    int64_t seq = 0;   // number of the last chunk readback enqueued (the mirror's last word once it has landed)
    dope::Img *dimg = nullptr;          // this context's descriptor (device)
    dope::Item *blk_items = nullptr, *chk_items = nullptr;
    dope::Queue *queue = nullptr;
    dope::Group grp{};                  // one-image launch group
    bool dirty = false;                 // device state advanced by a batch: refresh the host mirror
    int32_t lam_q8 = 0;
    bool energy_set = false;
    bool profiling = false;
    std::vector<hipEvent_t> ev_solve, ev_cons;   // start/stop pairs
    hipEvent_t ev_sync = nullptr;                // completion of the loop-control readback
    // A context over caller-provided device memory that may create nothing (solve_in_buffer): no events, no
    // pinned mirror (the loop control is copied back into hctl_host and the stream synchronised instead)
    bool no_alloc = false;
    Ctl hctl_host{};
    size_t n_solve = 0, n_cons = 0;
    std::string err;
};

namespace {

struct Layout {
    size_t ctl, img, bitems, citems, queue, btab, chunk, blist, u, w, cw, Y, A0, A1, yhat, yslot, resid, stats, labels,
        epart, axrow, gscr, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The max-flow solver takes the partition's blocks: in LDS, or in global memory for the stencils that have that
// solver.
bool maxflow_possible(const Geom &g) {
    return dope::maxflow_lds_bytes(g.max_np, g.hs) <= dope::MAXFLOW_LDS_LIMIT || g.max_np <= dope::gmem_max_np(g.conn);
}

// Per-block max-flow state in global memory when a block exceeds the LDS (0 otherwise).
size_t gmem_stride(const Geom &g) {
    const size_t b = dope::maxflow_lds_bytes(g.max_np, g.hs);
    return b > dope::MAXFLOW_LDS_LIMIT ? align256(b) : 0;
}


Layout layout_for(const Geom &g) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
    L.ctl = take(sizeof(Ctl));
    L.img = take(sizeof(dope::Img));
    L.bitems = take(size_t(g.K) * sizeof(dope::Item));
    const int64_t nbl = g.n - g.n_interior;   // boundary pixels
    L.citems = take(size_t((nbl + dope::CHUNK - 1) / dope::CHUNK) * sizeof(dope::Item));
    L.queue = take(sizeof(dope::Queue));
    L.btab = take(size_t(g.K) * dope::BTAB_STRIDE * 4);
    L.chunk = take(size_t((nbl + dope::CHUNK - 1) / dope::CHUNK) * 4);
    L.blist = take(size_t(nbl) * 8);
    L.u = take(size_t(g.n) * 4);
    L.w = take(size_t(g.n) * g.hs * 4);
    L.cw = take(size_t(g.n) * g.hs * 4);
    L.Y = take(size_t(g.n) * 4);
    L.A0 = take(size_t(g.tot) * 4);
    L.A1 = take(size_t(g.tot) * 4);
    L.yhat = take(size_t(g.tot));
    L.yslot = take(size_t(g.n) * dope::slot_count(g));
    L.resid = take(size_t(g.K) * 8);
    L.stats = take(size_t(g.K) * 16);
    L.labels = take(size_t(g.n));
    L.epart = take(size_t(dope::ENERGY_PARTS) * 8);
    L.axrow = take((size_t(g.W) + g.H + g.D) * 8);
    L.gscr = take(size_t(g.K) * gmem_stride(g));
    L.total = o;
    return L;
}

int half_stencil_size(int ndim, int conn) {
    if (ndim == 2 && conn == 4) return 2;
    if (ndim == 2 && conn == 8) return 4;
    if (ndim == 2 && conn == 24) return 12;   // 5x5 square neighbourhood
    if (ndim == 2 && conn == 48) return 24;   // 7x7 square neighbourhood
    if (ndim == 2 && conn == 80) return 40;   // 9x9 square neighbourhood
    if (ndim == 3 && conn == 6) return 3;
    if (ndim == 3 && conn == 32) return 16;   // ball of radius 2 (32 neighbours)
    if (ndim == 3 && conn == 122) return 61;  // ball of radius 3 (122 neighbours)
    if (ndim == 3 && conn == 256) return 128; // ball of radius 4 (256 neighbours)
    return 0;
}

int stencil_radius(int conn) {
    return (conn == 24 || conn == 32) ? 2 : ((conn == 48 || conn == 122) ? 3 : ((conn == 80 || conn == 256) ? 4 : 1));
}

// Builds the partition; returns an empty string on success or a message.
std::string make_geom(const dope_params *p, Geom &g, std::vector<int32_t> *btab) {
    if (!p) return "null params";
    if (p->ndim != 2 && p->ndim != 3) return "ndim must be 2 or 3";
    const int hs = half_stencil_size(p->ndim, p->connectivity);
    if (!hs) return "connectivity must be 4, 8, 24, 48 or 80 in 2D and 6, 32, 122 or 256 in 3D";
    int32_t dims[3] = {p->dims[0], p->dims[1], p->ndim == 3 ? p->dims[2] : 1};
    if (p->ndim == 2 && p->dims[2] != 1 && p->dims[2] != 0) return "dims[2] must be 1 in 2D";
    int64_t n = 1;
    for (int a = 0; a < 3; ++a) {
        if (dims[a] <= 0) return "dims must be positive";
        n *= dims[a];
    }
    // the kernels address per-pixel arrays with 32-bit byte offsets; the label slots take 4 (2D) or 8 (3D)
    // bytes per pixel
    if (n * (p->ndim == 3 ? 8 : 4) > (int64_t(1) << 32) - 1) return "grid too large (n must be < 2^30 in 2D, < 2^29 in 3D)";
    int64_t K = 1, max_np = 1;
    for (int a = 0; a < 3; ++a) {
        const int N = dims[a];
        const int B = (p->ndim == 2 && a == 2) ? 1 : p->block[a];
        const int o = (p->ndim == 2 && a == 2) ? 0 : p->overlap[a];
        dope::Axis ax;
        if (B <= 0 || B >= N) {
            ax = dope::make_axis(N, N, N, 1);
        } else {
            if (o < 0 || 2 * o > B) return "overlap must satisfy 0 <= o <= B/2";
            const int s = B - o;
            ax = dope::make_axis(N, B, s, 1 + (N - B + s - 1) / s);
        }
        g.ax[a] = ax;
        K *= ax.nb;
        max_np *= std::min(ax.B, N);
    }
    if (K >= (int64_t(1) << 28)) return "too many blocks";
    g.W = dims[0];
    g.H = dims[1];
    g.D = dims[2];
    g.conn = p->connectivity;
    g.hs = hs;
    g.rad = stencil_radius(p->connectivity);
    // the stencil must not reach past the neighbouring block: every offset changes the top block of a coordinate
    // by at most one
    for (int a = 0; a < 3; ++a)
        if (g.ax[a].nb > 1 && g.rad > g.ax[a].s) return "block stride B - o must be at least the stencil radius";
    g.K = int32_t(K);
    g.max_np = int32_t(max_np);
    g.n = n;
    int64_t tot = 0;
    if (btab) btab->assign(size_t(K) * dope::BTAB_STRIDE, 0);
    int64_t k = 0;
    for (int tz = 0; tz < g.ax[2].nb; ++tz)
        for (int ty = 0; ty < g.ax[1].nb; ++ty)
            for (int tx = 0; tx < g.ax[0].nb; ++tx, ++k) {
                const int x0 = tx * g.ax[0].s, y0 = ty * g.ax[1].s, z0 = tz * g.ax[2].s;
                const int ex = std::min(g.ax[0].B, g.W - x0), ey = std::min(g.ax[1].B, g.H - y0),
                          ez = std::min(g.ax[2].B, g.D - z0);
                if (btab) {
                    int32_t *r = btab->data() + k * dope::BTAB_STRIDE;
                    r[0] = x0; r[1] = y0; r[2] = z0; r[3] = ex; r[4] = ey; r[5] = ez; r[6] = int32_t(tot); r[7] = 0;
                }
                tot += int64_t(ex) * ey * ez;
                if (tot >= (int64_t(1) << 30)) return "sum of block sizes must be < 2^30";
            }
    g.tot = tot;
    for (int a = 0; a < 3; ++a)
        g.span[a] = int64_t(g.ax[a].nb - 1) * g.ax[a].B + dope::axis_ext(g.ax[a], g.ax[a].nb - 1);
    g.n_interior = 1;   // the interior rule is separable: product over axes of the interior counts
    for (int a = 0; a < 3; ++a) {
        const dope::Axis &ax = g.ax[a];
        int64_t cnt = 0;
        for (int t = 0; t < ax.nb; ++t)
            cnt += std::max(0, dope::axis_interior_hi(ax, t, g.rad) - dope::axis_interior_lo(ax, t, g.rad));
        g.n_interior *= cnt;
    }
    if (btab) {
        // the kernels locate blocks by the closed form; it must agree with the enumeration above
        int64_t kk = 0;
        for (int tz = 0; tz < g.ax[2].nb; ++tz)
            for (int ty = 0; ty < g.ax[1].nb; ++ty)
                for (int tx = 0; tx < g.ax[0].nb; ++tx, ++kk)
                    if (dope::block_offset(g, tx, ty, tz) != (*btab)[size_t(kk) * dope::BTAB_STRIDE + 6])
                        return "internal: block offset formula disagrees with the partition";
    }
    {
        // one-image block solves take their block from the dispatch order: a permutation of the blocks
        std::vector<uint8_t> seen(size_t(g.K), 0);
        for (int32_t b = 0; b < g.K; ++b) {
            const int32_t k = dope::block_at(g, b);
            if (k < 0 || k >= g.K || seen[size_t(k)]) return "internal: block dispatch order is not a permutation";
            seen[size_t(k)] = 1;
        }
    }
    if (p->mu0 < 1 || p->mu0 > dope::MU_MAX) return "mu0 must be in [1, 2^24 - 1]";
    if (p->mu_fact_num < 0 || p->mu_fact_den < 0) return "mu_fact must be positive";
    if ((p->mu_fact_num == 0) != (p->mu_fact_den == 0)) return "mu_fact numerator and denominator must both be set";
    if (p->eps_q16 < 0) return "eps_q16 must be >= 0";
    if (p->max_iter < 0) return "max_iter must be >= 0";
    // blocks beyond the LDS take the global-memory solver (at most 16384 pixels with the 3x3 stencils, 4096 with
    // the wide ones)
    const bool maxflow_ok = dope::maxflow_lds_bytes(g.max_np, hs) <= dope::MAXFLOW_LDS_LIMIT ||
                            g.max_np <= dope::gmem_max_np(p->connectivity);
    const std::string too_big_msg = "block too large for the max-flow solver: more than " +
                                    std::to_string(dope::gmem_max_np(p->connectivity)) + " pixels beyond the LDS";
    const char *too_big = too_big_msg.c_str();
    switch (p->solver) {
        case DOPE_SOLVER_MAXFLOW:
            if (!maxflow_ok) return too_big;
            break;
        case DOPE_SOLVER_EXHAUSTIVE:
            if (g.max_np > 16) return "the exhaustive solver needs blocks of at most 16 pixels";
            break;
        case DOPE_SOLVER_LSATR:
            if (p->connectivity != 4 && p->connectivity != 8 && p->connectivity != 6)
                return "the LSA-TR solver takes the 4-, 8- and 6-connected stencils";
            if (dope::lsatr_lds_bytes(g.max_np, hs) > dope::LDS_LIMIT - 64 || g.max_np > dope::LSATR_MAX_NP)
                return "block too large for the LSA-TR solver (its state must fit the LDS)";
            break;
        case DOPE_SOLVER_AUTO:
            if (!maxflow_ok && g.max_np > 16) return too_big;
            break;
        default:
            return "unknown solver";
    }
    return std::string();
}

thread_local std::string g_create_error;

// The boundary list (the consensus kernel's work; interior copies are finished by the block-solve kernel) holds
// (block-major index, block) of the owner copy of every pixel that is not interior to its block, block by block
// and in each block's local raster order; the owner copy is the one in the block with the highest index along
// every axis.  The host computes, per block, how many such pixels it owns (a closed form: the owned box minus the
// interior box) and where its entries start (btab[k][7]); the device writes the entries (launch_build_blist).
// chunk: block of the first entry of every CHUNK entries.  Every block owns at least one such pixel when there
// are two or more blocks, so the owners within a chunk are consecutive block indices (checked).
bool build_tables(const Geom &g, std::vector<int32_t> &btab, int64_t &nbl, std::vector<int32_t> &chunk) {
    nbl = 0;
    chunk.clear();
    int64_t k = 0;
    for (int tz = 0; tz < g.ax[2].nb; ++tz)
        for (int ty = 0; ty < g.ax[1].nb; ++ty)
            for (int tx = 0; tx < g.ax[0].nb; ++tx, ++k) {
                const int t[3] = {tx, ty, tz};
                int64_t owned = 1, inner = 1;
                for (int a = 0; a < 3; ++a) {
                    const dope::Axis &ax = g.ax[a];
                    const int32_t start = t[a] * ax.s;
                    const int32_t olen = t[a] < ax.nb - 1 ? ax.s : ax.N - start;
                    const int32_t ilen = std::max(0, dope::axis_interior_hi(ax, t[a], g.rad) -
                                                         dope::axis_interior_lo(ax, t[a], g.rad));
                    owned *= olen;
                    inner *= ilen;
                }
                const int64_t cnt = owned - inner;
                if (g.K > 1 && cnt < 1) return false;
                btab[size_t(k) * dope::BTAB_STRIDE + 7] = int32_t(nbl);
                for (int64_t e = (nbl + dope::CHUNK - 1) / dope::CHUNK * dope::CHUNK; e < nbl + cnt; e += dope::CHUNK)
                    chunk.push_back(int32_t(k));
                nbl += cnt;
            }
    return nbl == g.n - g.n_interior;
}

dope_status fail(dope_ctx *c, dope_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

dope_status hip_fail(dope_ctx *c, hipError_t e, const char *what) {
    return fail(c, DOPE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                        \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

void assign_pointers(dope_ctx *c) {
    const Layout L = layout_for(c->g);
    char *b = c->ws;
    c->ctl = reinterpret_cast<Ctl *>(b + L.ctl);
    c->btab = reinterpret_cast<int32_t *>(b + L.btab);
    c->chunk_k0 = reinterpret_cast<int32_t *>(b + L.chunk);
    c->blist = reinterpret_cast<int2 *>(b + L.blist);
    c->dimg = reinterpret_cast<dope::Img *>(b + L.img);
    c->blk_items = reinterpret_cast<dope::Item *>(b + L.bitems);
    c->chk_items = reinterpret_cast<dope::Item *>(b + L.citems);
    c->queue = reinterpret_cast<dope::Queue *>(b + L.queue);
    c->u = reinterpret_cast<int32_t *>(b + L.u);
    c->w = reinterpret_cast<int32_t *>(b + L.w);
    c->cw = reinterpret_cast<int32_t *>(b + L.cw);
    c->Y = reinterpret_cast<int32_t *>(b + L.Y);
    c->A0 = reinterpret_cast<int32_t *>(b + L.A0);
    c->A1 = reinterpret_cast<int32_t *>(b + L.A1);
    c->yhat = reinterpret_cast<uint8_t *>(b + L.yhat);
    c->yslot = reinterpret_cast<uint8_t *>(b + L.yslot);
    c->resid = reinterpret_cast<int64_t *>(b + L.resid);
    c->stats = reinterpret_cast<int32_t *>(b + L.stats);
    c->labels = reinterpret_cast<uint8_t *>(b + L.labels);
    c->epart = reinterpret_cast<int64_t *>(b + L.epart);
    c->axrow = reinterpret_cast<int2 *>(b + L.axrow);
    c->gscr = gmem_stride(c->g) ? reinterpret_cast<unsigned char *>(b + L.gscr) : nullptr;
}

dope::Img host_img(const dope_ctx *c) {
    dope::Img im{};
    im.g = c->g;
    im.u = c->u;
    im.w = c->w;
    im.cw = c->cw;
    im.btab = c->btab;
    im.chunk_k0 = c->chunk_k0;
    im.blist = c->blist;
    im.Y = c->Y;
    im.A0 = c->A0;
    im.A1 = c->A1;
    im.stats = c->stats;
    im.yhat = c->yhat;
    im.yslot = c->yslot;
    im.resid = c->resid;
    im.ctl = c->ctl;
    im.summary = nullptr;
    im.axrow = c->axrow;
    im.n_chunks = int32_t(c->hchunk.size());
    im.n_blist = int32_t(c->nbl);
    return im;
}

dope_status upload_tables(dope_ctx *c) {
    HIP_TRY(c, hipMemcpyAsync(c->btab, c->hbtab.data(), c->hbtab.size() * 4, hipMemcpyHostToDevice, c->stream),
            "block table upload");
    if (!c->hchunk.empty())
        HIP_TRY(c, hipMemcpyAsync(c->chunk_k0, c->hchunk.data(), c->hchunk.size() * 4, hipMemcpyHostToDevice,
                                  c->stream), "chunk table upload");
    if (c->nbl > 0) HIP_TRY(c, dope::launch_build_blist(c->g, c->btab, c->blist, c->stream), "boundary list");
    HIP_TRY(c, dope::launch_axis_rows(c->g, c->axrow, c->stream), "axis rows");
    // one-image launch group: descriptor, work items, zeroed queue (staged in host memory that stays alive
    // until the synchronisation at the end of this function)
    const dope::Img im = host_img(c);
    c->himg = im;
    std::vector<dope::Item> bi(size_t(c->g.K)), ci(c->hchunk.size());
    for (size_t k = 0; k < bi.size(); ++k) bi[k] = dope::Item{0, int32_t(k)};
    for (size_t k = 0; k < ci.size(); ++k) ci[k] = dope::Item{0, int32_t(k)};
    const dope::Queue q{};
    HIP_TRY(c, hipMemcpyAsync(c->dimg, &im, sizeof(im), hipMemcpyHostToDevice, c->stream), "descriptor upload");
    HIP_TRY(c, hipMemcpyAsync(c->blk_items, bi.data(), bi.size() * sizeof(dope::Item), hipMemcpyHostToDevice,
                              c->stream), "item upload");
    if (!ci.empty())
        HIP_TRY(c, hipMemcpyAsync(c->chk_items, ci.data(), ci.size() * sizeof(dope::Item), hipMemcpyHostToDevice,
                                  c->stream), "item upload");
    HIP_TRY(c, hipMemcpyAsync(c->queue, &q, sizeof(q), hipMemcpyHostToDevice, c->stream), "queue upload");
    // a zeroed loop control: the setup kernel initialises every field except the validation accumulator
    const dope::Ctl zc{};
    c->ctl_fresh = false;
    HIP_TRY(c, hipMemcpyAsync(c->ctl, &zc, sizeof(zc), hipMemcpyHostToDevice, c->stream), "control reset");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    c->grp = dope::Group{c->dimg, 1, c->blk_items, c->g.K, c->chk_items, int32_t(ci.size()), c->queue,
                         c->g.conn, 0, c->g.max_np, 0};
    c->grp.gscratch = c->gscr;
    c->grp.gstride = gmem_stride(c->g);
    return DOPE_OK;
}

dope_status ensure_workspace(dope_ctx *c) {
    if (c->ws) return DOPE_OK;
    const size_t bytes = layout_for(c->g).total;
    void *ptr = nullptr;
    if (hipMalloc(&ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DOPE_ENOMEM, "hipMalloc of the workspace failed");
    }
    c->ws = static_cast<char *>(ptr);
    c->ws_bytes = bytes;
    c->own_ws = true;
    assign_pointers(c);
    return upload_tables(c);
}

// Waits for the work enqueued on the context stream.  The loop-control readback sits on the critical path of
// every solve, so the host polls a completion event for up to ~2 ms before it blocks: a blocking wait adds the
// wake-up latency of the host thread to every readback.
dope_status wait_stream(dope_ctx *c) {
    if (c->no_alloc) {
        HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
        return DOPE_OK;
    }
    if (!c->ev_sync && hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming) != hipSuccess) {
        c->ev_sync = nullptr;
        HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
        return DOPE_OK;
    }
    HIP_TRY(c, hipEventRecord(c->ev_sync, c->stream), "event record");
    for (int spin = 0; spin < 200000; ++spin) {
        const hipError_t q = hipEventQuery(c->ev_sync);
        if (q == hipSuccess) return DOPE_OK;
        if (q != hipErrorNotReady) return hip_fail(c, q, "event query");
        if (spin > 20000) break;
    }
    HIP_TRY(c, hipEventSynchronize(c->ev_sync), "event synchronize");
    return DOPE_OK;
}

// Waits for the mirror of the chunk enqueued last: its loop-control kernel writes the mirror and then, with
// system-scope release, the chunk's readback number; polling that word returns as soon as it lands, ahead of the
// kernel's completion signal.  A chunk still running after a few milliseconds falls back to the stream event,
// which also reports a failed kernel.
dope_status wait_mirror(dope_ctx *c) {
    const int64_t want = c->seq;
    const auto t0 = std::chrono::steady_clock::now();
    for (int spin = 0;; ++spin) {
        if (__atomic_load_n(&c->hctl->seq, __ATOMIC_ACQUIRE) == want) return DOPE_OK;
        if ((spin & 255) == 255 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
    }
    dope_status st = wait_stream(c);
    if (st != DOPE_OK) return st;
    if (__atomic_load_n(&c->hctl->seq, __ATOMIC_ACQUIRE) != want)
        return fail(c, DOPE_EDEVICE, "loop-control readback: the mirror was not written");
    return DOPE_OK;
}

dope_status sync_ctl(dope_ctx *c) {
    // a pending energy validation is taken before the loop control is read back
    if (c->validate_pending) {
        HIP_TRY(c, dope::launch_validate(c->ctl, c->stream), "validation launch");
        c->validate_pending = false;
    }
    // the readback number is the host's own (the device never writes it in the control block): not copied
    HIP_TRY(c, hipMemcpyAsync(c->hctl, c->ctl, offsetof(Ctl, seq), hipMemcpyDeviceToHost, c->stream),
            "control readback");
    return wait_stream(c);
}

void fill_info(const dope_ctx *c, dope_info *out) {
    if (!out) return;
    out->iters_done = c->hctl->t;
    out->converged = c->hctl->converged;
    out->max_resid2 = int64_t(c->hctl->last_max_resid);
    out->mu = c->hctl->M;
}

hipEvent_t next_event(std::vector<hipEvent_t> &pool, size_t idx) {
    while (pool.size() <= idx) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back(e);
    }
    return pool[idx];
}

// Enqueues count iterations after the c->hctl->t completed ones (the host mirror is current whenever this runs).
// The last iteration's loop-control kernel also refreshes the pinned host mirror, so the readback that follows is
// a wait on the stream instead of a copy launch (see read_back).
dope_status enqueue_iterations(dope_ctx *c, int count) {
    c->grp.solver = c->solver;
    c->grp.one = &c->himg;
    for (int it = 0; it < count; ++it) {
        c->grp.par = (c->hctl->t + it) & 1;
        Ctl *mirror = (it == count - 1 && !c->no_alloc) ? c->hctl : nullptr;
        const int64_t seq = mirror ? ++c->seq : 0;
        if (!c->profiling) {
            HIP_TRY(c, dope::launch_iteration(c->grp, c->stream, mirror, seq), "iteration launch");
            continue;
        }
        hipEvent_t e0 = next_event(c->ev_solve, 2 * c->n_solve), e1 = next_event(c->ev_solve, 2 * c->n_solve + 1);
        HIP_TRY(c, dope::launch_solve_phase(c->grp, c->stream, e0 && e1 ? e0 : nullptr, e0 && e1 ? e1 : nullptr),
                "block solve launch");
        if (e0 && e1) ++c->n_solve;
        e0 = next_event(c->ev_cons, 2 * c->n_cons);
        e1 = next_event(c->ev_cons, 2 * c->n_cons + 1);
        HIP_TRY(c, dope::launch_consensus_phase(c->grp, c->stream, e0 && e1 ? e0 : nullptr, e0 && e1 ? e1 : nullptr),
                "consensus launch");
        if (e0 && e1 && c->grp.n_chk_items > 0) ++c->n_cons;
        HIP_TRY(c, dope::launch_finalize_phase(c->grp, c->stream, mirror, seq), "finalize launch");
    }
    return DOPE_OK;
}

// The loop control after enqueue_iterations(c, count): the mirror is written by the last loop-control kernel when
// count > 0 (contexts with a pinned mirror), otherwise it is copied back.
dope_status read_back(dope_ctx *c, int count) {
    return (count > 0 && !c->no_alloc) ? wait_mirror(c) : sync_ctl(c);
}

dope_status check_ready(dope_ctx *c) {
    if (!c) return DOPE_EINVAL;
    if (!c->energy_set) return fail(c, DOPE_ESTATE, "dope_set_energy has not been called");
    if (c->dirty) {
        c->dirty = false;
        return sync_ctl(c);
    }
    return DOPE_OK;
}

}  // namespace

extern "C" {

dope_status dope_create(const dope_params *p, dope_ctx **out) {
    if (!out) return DOPE_EINVAL;
    *out = nullptr;
    Geom g{};
    std::vector<int32_t> bt;
    dope_params q = p ? *p : dope_params{};
    if (p && q.mu_fact_num == 0 && q.mu_fact_den == 0) { q.mu_fact_num = 21; q.mu_fact_den = 20; }
    const std::string msg = make_geom(p ? &q : nullptr, g, &bt);
    g_create_error = msg;
    if (!msg.empty()) return DOPE_EINVAL;
    dope_ctx *c = new (std::nothrow) dope_ctx();
    if (!c) return DOPE_ENOMEM;
    c->p = q;
    c->g = g;
    c->hbtab.swap(bt);
    if (!build_tables(c->g, c->hbtab, c->nbl, c->hchunk)) {
        g_create_error = "internal: boundary pixel table inconsistent with the partition";
        delete c;
        return DOPE_EINVAL;
    }
    if (q.stream) {
        c->stream = static_cast<hipStream_t>(q.stream);
    } else {
        // a blocking stream: ordered with work that PyTorch issues on the default stream
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return DOPE_EDEVICE;
        }
        c->own_stream = true;
    }
    void *h = nullptr;
    if (hipHostMalloc(&h, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return DOPE_EDEVICE;
    }
    c->hctl = static_cast<Ctl *>(h);
    std::memset(c->hctl, 0, sizeof(Ctl));
    *out = c;
    return DOPE_OK;
}

dope_status dope_autotune(int32_t ndim, const int32_t dims[3], int32_t connectivity, int32_t block[3],
                          int32_t overlap[3]) {
    if (!dims || !block || !overlap) return DOPE_EINVAL;
    if (!half_stencil_size(ndim, connectivity)) return DOPE_EINVAL;
    // the row of the measured image size nearest to the shorter side (table written by the offline sweep)
    int32_t short_side = std::min(dims[0], dims[1]);
    if (ndim == 3) short_side = std::min(short_side, dims[2]);
    for (const dope::TuneRow &r : dope::TUNE_TABLE) {
        if (r.ndim != ndim || r.conn != connectivity || short_side > r.max_short_side) continue;
        for (int a = 0; a < 3; ++a) {
            const bool on = a < ndim;
            block[a] = on ? r.block : 1;
            overlap[a] = on ? r.overlap : 0;
        }
        return DOPE_OK;
    }
    if (ndim == 3 && connectivity == 256) {
        // the radius-4 ball (not in the sweep): its 1065 LDS bytes per node allow 5^3 blocks, stride 4 = radius
        for (int a = 0; a < 3; ++a) { block[a] = 5; overlap[a] = 1; }
        return DOPE_OK;
    }
    return DOPE_EINVAL;
}

size_t dope_workspace_bytes(const dope_params *p) {
    Geom g{};
    if (!p) return 0;
    dope_params q = *p;
    if (q.mu_fact_num == 0 && q.mu_fact_den == 0) { q.mu_fact_num = 21; q.mu_fact_den = 20; }
    if (!make_geom(&q, g, nullptr).empty()) return 0;
    return layout_for(g).total;
}

dope_status dope_dispatch_order(const dope_params *p, int32_t *n_blocks, int32_t *order) {
    Geom g{};
    if (!p || !n_blocks) {
        g_create_error = "null params or n_blocks";
        return DOPE_EINVAL;
    }
    dope_params q = *p;
    if (q.mu_fact_num == 0 && q.mu_fact_den == 0) { q.mu_fact_num = 21; q.mu_fact_den = 20; }
    g_create_error = make_geom(&q, g, nullptr);
    if (!g_create_error.empty()) return DOPE_EINVAL;
    *n_blocks = g.K;
    if (order)
        for (int32_t b = 0; b < g.K; ++b) order[b] = dope::block_at(g, b);
    return DOPE_OK;
}

dope_status dope_bind_workspace(dope_ctx *c, void *dev_ptr, size_t bytes) {
    if (!c || !dev_ptr) return DOPE_EINVAL;
    if (c->ws) return fail(c, DOPE_ESTATE, "a workspace is already in use");
    if (reinterpret_cast<uintptr_t>(dev_ptr) & 255) return fail(c, DOPE_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < layout_for(c->g).total) return fail(c, DOPE_ENOMEM, "workspace smaller than dope_workspace_bytes");
    c->ws = static_cast<char *>(dev_ptr);
    c->ws_bytes = bytes;
    c->own_ws = false;
    assign_pointers(c);
    return upload_tables(c);
}

}  // extern "C"

namespace {

// Copies u and w, resets the state and enqueues the weight preparation and validation; no synchronisation.
dope_status enqueue_energy(dope_ctx *c, const int32_t *u, const int32_t *w, int32_t lambda_q8, int32_t mem_kind,
                           int32_t allow_negative) {
    if (!c || !u || !w) return DOPE_EINVAL;
    if (lambda_q8 < 0) return fail(c, DOPE_EINVAL, "lambda must be >= 0");
    if (mem_kind != DOPE_MEM_HOST && mem_kind != DOPE_MEM_DEVICE) return fail(c, DOPE_EINVAL, "bad mem_kind");
    dope_status st = ensure_workspace(c);
    if (st != DOPE_OK) return st;
    const Geom &g = c->g;
    // host inputs are uploaded into the workspace (w only as staging for the setup kernel); device inputs are read
    // by the setup kernel directly
    const int32_t *u_src = u, *w_src = w;
    if (mem_kind == DOPE_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(c->u, u, size_t(g.n) * 4, hipMemcpyHostToDevice, c->stream), "unary upload");
        HIP_TRY(c, hipMemcpyAsync(c->w, w, size_t(g.n) * g.hs * 4, hipMemcpyHostToDevice, c->stream), "weight upload");
        u_src = c->u;
        w_src = c->w;
    }
    const uint64_t eps2 = uint64_t(c->p.eps_q16) * uint64_t(c->p.eps_q16);
    // a verdict still pending (an earlier set-up no call has run since) consumes its bits first, so that they do
    // not reach this one's
    if (c->validate_pending) HIP_TRY(c, dope::launch_validate(c->ctl, c->stream), "validation launch");
    HIP_TRY(c, dope::launch_setup(g, u_src, w_src, c->u, c->cw, lambda_q8, c->Y, c->A0, c->A1, c->yhat, c->resid,
                                  c->ctl, c->p.mu0, c->p.mu_fact_num, c->p.mu_fact_den, eps2, allow_negative,
                                  c->p.max_iter, c->stream),
            "setup launch");
    c->validate_pending = true;
    c->ctl_fresh = true;
    return DOPE_OK;
}

const char *status_message(int32_t status, int32_t flags) {
    switch (status) {
        case DOPE_EOVERFLOW: return "fixed-point overflow (|Y| or |A| >= 2^22): mu too small";
        case DOPE_ESOLVER: return "block max-flow exceeded its round limit";
        case DOPE_ENOTSUBMODULAR: return "negative weight with the max-flow solver";
        case DOPE_EINVAL:
            return (flags & dope::FLAG_OFFGRID) ? "nonzero weight on an off-grid edge"
                                                : "weights too large: per-node sum |c_ij| >= 2^29";
        default: return "error";
    }
}

}  // namespace

extern "C" {

dope_status dope_set_energy(dope_ctx *c, const int32_t *u, const int32_t *w, int32_t lambda_q8, int32_t mem_kind) {
    if (!c) return DOPE_EINVAL;
    c->energy_set = false;
    dope_status st = enqueue_energy(c, u, w, lambda_q8, mem_kind, c->p.solver != DOPE_SOLVER_MAXFLOW);
    if (st != DOPE_OK) return st;
    c->dirty = false;
    st = sync_ctl(c);
    if (st != DOPE_OK) return st;
    const Geom &g = c->g;
    const int32_t flags = c->hctl->vflags;
    if (flags & dope::FLAG_OFFGRID) return fail(c, DOPE_EINVAL, "nonzero weight on an off-grid edge");
    if (flags & dope::FLAG_TOOBIG) return fail(c, DOPE_EINVAL, "weights too large: per-node sum |c_ij| >= 2^29");
    int solver = c->p.solver;
    if (flags & dope::FLAG_NEGATIVE) {
        if (solver == DOPE_SOLVER_MAXFLOW) return fail(c, DOPE_ENOTSUBMODULAR, "negative weight with the max-flow solver");
        if (solver == DOPE_SOLVER_AUTO) {
            if (g.max_np > 16) return fail(c, DOPE_ENOTSUBMODULAR, "negative weight and blocks too large to enumerate");
            solver = DOPE_SOLVER_EXHAUSTIVE;
        }
    } else if (solver == DOPE_SOLVER_AUTO) {
        solver = maxflow_possible(g) ? DOPE_SOLVER_MAXFLOW : DOPE_SOLVER_EXHAUSTIVE;
    }
    c->solver = solver;
    c->lam_q8 = lambda_q8;
    c->energy_set = true;
    c->err.clear();
    return DOPE_OK;
}

dope_status dope_set_energy_async(dope_ctx *c, const int32_t *u, const int32_t *w, int32_t lambda_q8,
                                  int32_t mem_kind) {
    if (!c) return DOPE_EINVAL;
    int solver = c->p.solver;
    if (solver == DOPE_SOLVER_AUTO)
        solver = maxflow_possible(c->g) ? DOPE_SOLVER_MAXFLOW : DOPE_SOLVER_EXHAUSTIVE;
    c->energy_set = false;
    dope_status st = enqueue_energy(c, u, w, lambda_q8, mem_kind, solver != DOPE_SOLVER_MAXFLOW);
    if (st != DOPE_OK) return st;
    // host mirror of the reset state; a validation failure shows up at the next readback
    Ctl h{};
    h.t_limit = c->p.max_iter;
    h.stop_on_converge = 1;
    h.M = c->p.mu0;
    h.eps2 = uint64_t(c->p.eps_q16) * uint64_t(c->p.eps_q16);
    h.mu_num = c->p.mu_fact_num;
    h.mu_den = c->p.mu_fact_den;
    *c->hctl = h;
    c->dirty = false;
    c->solver = solver;
    c->lam_q8 = lambda_q8;
    c->energy_set = true;
    c->err.clear();
    return DOPE_OK;
}

dope_status dope_iterate(dope_ctx *c, int32_t n_iter, dope_info *out) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (n_iter < 0) return fail(c, DOPE_EINVAL, "n_iter must be >= 0");
    if (c->hctl->status != 0) { fill_info(c, out); return dope_status(c->hctl->status); }
    const int32_t t0 = c->hctl->t;
    HIP_TRY(c, dope::launch_ctl_setup(c->ctl, t0 + n_iter, 0, 0, c->stream), "control setup launch");
    c->validate_pending = false;
    c->ctl_fresh = false;
    st = enqueue_iterations(c, n_iter);
    if (st != DOPE_OK) return st;
    st = read_back(c, n_iter);
    if (st != DOPE_OK) return st;
    fill_info(c, out);
    if (c->hctl->status != 0)
        return fail(c, dope_status(c->hctl->status), status_message(c->hctl->status, c->hctl->vflags));
    return DOPE_OK;
}

dope_status dope_solve(dope_ctx *c, dope_info *out) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (c->hctl->status != 0) { fill_info(c, out); return dope_status(c->hctl->status); }
    if (c->hctl->t > 0 && c->hctl->converged) { fill_info(c, out); return DOPE_OK; }
    const int32_t limit = c->p.max_iter;
    if (c->hctl->t >= limit) {
        // no iteration to run (max_iter = 0, or t already at the cap): a pending verdict is taken and the loop
        // control read back, so a rejected energy is reported here and its bits do not reach the next upload
        c->ctl_fresh = false;
        st = sync_ctl(c);
        if (st != DOPE_OK) return st;
        fill_info(c, out);
        if (c->hctl->status != 0)
            return fail(c, dope_status(c->hctl->status), status_message(c->hctl->status, c->hctl->vflags));
        return DOPE_OK;
    }
    if (!c->ctl_fresh) HIP_TRY(c, dope::launch_ctl_setup(c->ctl, limit, 1, 0, c->stream), "control setup launch");
    c->validate_pending = false;
    c->ctl_fresh = false;
    // Iterations are enqueued in chunks of 2, 2, 4, 8, ... with one readback per chunk.  An iteration enqueued
    // after the stopping rule held is skipped on the device (Ctl::halted), so the result is that of one
    // iteration per readback; only a few empty launches are spent.
    int chunk = 2, n_chunks = 0;
    while (c->hctl->t < limit) {
        const int count = std::min(chunk, limit - c->hctl->t);
        st = enqueue_iterations(c, count);
        if (st != DOPE_OK) return st;
        st = read_back(c, count);
        if (st != DOPE_OK) return st;
        if (c->hctl->halted) break;
        if (++n_chunks >= 2) chunk = std::min(2 * chunk, 64);
    }
    fill_info(c, out);
    if (c->hctl->status != 0)
        return fail(c, dope_status(c->hctl->status), status_message(c->hctl->status, c->hctl->vflags));
    return DOPE_OK;
}

dope_status dope_labels(dope_ctx *c, uint8_t *labels, int32_t mem_kind) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (!labels) return fail(c, DOPE_EINVAL, "null labels");
    uint8_t *dst = mem_kind == DOPE_MEM_DEVICE ? labels : c->labels;
    HIP_TRY(c, dope::launch_labels(c->g, c->Y, dst, c->stream), "labels launch");
    if (mem_kind == DOPE_MEM_DEVICE) return DOPE_OK;    // stream-ordered, no wait
    HIP_TRY(c, hipMemcpyAsync(labels, c->labels, size_t(c->g.n), hipMemcpyDeviceToHost, c->stream), "labels copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return DOPE_OK;
}

dope_status dope_energy(dope_ctx *c, int64_t *e_q8) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (!e_q8) return fail(c, DOPE_EINVAL, "null output");
    HIP_TRY(c, dope::launch_energy(c->g, c->u, c->cw, c->Y, c->epart, c->ctl, c->stream), "energy launch");
    st = sync_ctl(c);
    if (st != DOPE_OK) return st;
    // the pairwise term is recovered from c_ij, which a rejected energy does not hold in full
    if (c->hctl->status == DOPE_EINVAL)
        return fail(c, DOPE_EINVAL, status_message(c->hctl->status, c->hctl->vflags));
    *e_q8 = c->hctl->energy;
    return DOPE_OK;
}

dope_status dope_get_state(dope_ctx *c, int32_t *Y, int32_t *A, uint8_t *yhat, int64_t *mu, int32_t *t) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    st = sync_ctl(c);
    if (st != DOPE_OK) return st;
    const Geom &g = c->g;
    const int32_t *Acur = (c->hctl->t & 1) ? c->A1 : c->A0;
    if (Y) HIP_TRY(c, hipMemcpyAsync(Y, c->Y, size_t(g.n) * 4, hipMemcpyDeviceToHost, c->stream), "Y copy");
    if (A) HIP_TRY(c, hipMemcpyAsync(A, Acur, size_t(g.tot) * 4, hipMemcpyDeviceToHost, c->stream), "A copy");
    if (yhat) HIP_TRY(c, hipMemcpyAsync(yhat, c->yhat, size_t(g.tot), hipMemcpyDeviceToHost, c->stream), "yhat copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (mu) *mu = c->hctl->M;
    if (t) *t = c->hctl->t;
    return DOPE_OK;
}

dope_status dope_set_state(dope_ctx *c, const int32_t *Y, const int32_t *A, const uint8_t *yhat, int64_t mu,
                           int32_t t) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (!Y || !A || !yhat) return fail(c, DOPE_EINVAL, "null state array");
    if (mu < 1 || mu > dope::MU_MAX || t < 0) return fail(c, DOPE_EINVAL, "bad mu or t");
    const Geom &g = c->g;
    for (int64_t i = 0; i < g.n; ++i)
        if (Y[i] >= dope::STATE_LIMIT || Y[i] <= -dope::STATE_LIMIT) return fail(c, DOPE_EINVAL, "Y out of range");
    for (int64_t i = 0; i < g.tot; ++i)
        if (A[i] >= dope::STATE_LIMIT || A[i] <= -dope::STATE_LIMIT) return fail(c, DOPE_EINVAL, "A out of range");
    st = sync_ctl(c);
    if (st != DOPE_OK) return st;
    int32_t *Acur = (t & 1) ? c->A1 : c->A0;
    HIP_TRY(c, hipMemcpyAsync(c->Y, Y, size_t(g.n) * 4, hipMemcpyHostToDevice, c->stream), "Y upload");
    HIP_TRY(c, hipMemcpyAsync(Acur, A, size_t(g.tot) * 4, hipMemcpyHostToDevice, c->stream), "A upload");
    HIP_TRY(c, hipMemcpyAsync(c->yhat, yhat, size_t(g.tot), hipMemcpyHostToDevice, c->stream), "yhat upload");
    Ctl h = *c->hctl;
    h.M = mu;
    h.t = t;
    h.t_limit = t;
    h.halted = 0;
    h.status = 0;
    h.converged = 0;
    h.max_resid = 0;
    h.last_max_resid = 0;
    h.ovf_pending = 0;
    h.solver_err = 0;
    h.wg_counter = 0;
    *c->hctl = h;
    c->ctl_fresh = false;
    HIP_TRY(c, hipMemcpyAsync(c->ctl, c->hctl, offsetof(Ctl, seq), hipMemcpyHostToDevice, c->stream),
            "control upload");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return DOPE_OK;
}

dope_status dope_block_resid(dope_ctx *c, int64_t *resid) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (!resid) return fail(c, DOPE_EINVAL, "null output");
    HIP_TRY(c, hipMemcpyAsync(resid, c->resid, size_t(c->g.K) * 8, hipMemcpyDeviceToHost, c->stream), "resid copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return DOPE_OK;
}

dope_status dope_block_stats(dope_ctx *c, int32_t *stats) {
    dope_status st = check_ready(c);
    if (st != DOPE_OK) return st;
    if (!stats) return fail(c, DOPE_EINVAL, "null output");
    HIP_TRY(c, hipMemcpyAsync(stats, c->stats, size_t(c->g.K) * 16, hipMemcpyDeviceToHost, c->stream), "stats copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return DOPE_OK;
}

dope_status dope_block_table(dope_ctx *c, int32_t *n_blocks, int32_t *table) {
    if (!c || !n_blocks) return DOPE_EINVAL;
    *n_blocks = c->g.K;
    if (table)
        for (int64_t k = 0; k < c->g.K; ++k)
            std::memcpy(table + 7 * k, c->hbtab.data() + dope::BTAB_STRIDE * k, 7 * sizeof(int32_t));
    return DOPE_OK;
}

dope_status dope_sizes(const dope_ctx *c, int64_t *n, int32_t *n_blocks, int64_t *total_block_px, int32_t *h) {
    if (!c) return DOPE_EINVAL;
    if (n) *n = c->g.n;
    if (n_blocks) *n_blocks = c->g.K;
    if (total_block_px) *total_block_px = c->g.tot;
    if (h) *h = c->g.hs;
    return DOPE_OK;
}

dope_status dope_profile_enable(dope_ctx *c, int32_t on) {
    if (!c) return DOPE_EINVAL;
    c->profiling = on != 0;
    c->n_solve = c->n_cons = 0;
    return DOPE_OK;
}

dope_status dope_profile_read(dope_ctx *c, double *solve_ms, int32_t *solve_launches, double *consensus_ms,
                              int32_t *consensus_launches) {
    if (!c) return DOPE_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
    double ts = 0, tc = 0;
    for (size_t i = 0; i < c->n_solve; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, c->ev_solve[2 * i], c->ev_solve[2 * i + 1]) == hipSuccess) ts += ms;
    }
    for (size_t i = 0; i < c->n_cons; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, c->ev_cons[2 * i], c->ev_cons[2 * i + 1]) == hipSuccess) tc += ms;
    }
    if (solve_ms) *solve_ms = ts;
    if (solve_launches) *solve_launches = int32_t(c->n_solve);
    if (consensus_ms) *consensus_ms = tc;
    if (consensus_launches) *consensus_launches = int32_t(c->n_cons);
    return DOPE_OK;
}

const char *dope_last_error(const dope_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void dope_destroy(dope_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->ev_sync) (void)hipEventDestroy(c->ev_sync);
    for (hipEvent_t e : c->ev_solve) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_cons) (void)hipEventDestroy(e);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->hctl) (void)hipHostFree(c->hctl);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------------------
// Batches
// ------------------------------------------------------------------------------------------------------------

struct dope_batch {
    std::vector<dope_ctx *> ctxs;
    hipStream_t stream = nullptr;
    char *dbuf = nullptr;
    size_t dcap = 0, hcap = 0;     // capacities of dbuf (bytes) and of the pinned arrays (images)
    dope::Img *imgs = nullptr;
    int32_t *dsum = nullptr, *dparams = nullptr;
    dope::Group grp{};
    int32_t *hsum = nullptr;       // pinned: {t, halted, converged, status} per image
    int32_t *hparams = nullptr;    // pinned: {t_limit, stop} per image
    bool use_graph = false, graph_ready = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_sync = nullptr;   // completion of the summary readback
    // batched energy upload and labels: (image, pixel row) items, per-image arguments and label pointers
    dope::Item *rows = nullptr;
    int32_t n_rows = 0;
    dope::SetupArg *dargs = nullptr, *hargs = nullptr;   // device / pinned staging
    uint8_t **dlabs = nullptr, **hlabs = nullptr;         // device / pinned staging
    hipEvent_t ev_stage = nullptr;   // the last upload of the pinned staging arrays has run after this
    std::string err;
};

namespace {

dope_status bfail(dope_batch *b, dope_status s, const std::string &msg) {
    if (b) b->err = msg;
    return s;
}

#define BHIP_TRY(b, expr, what)                                                                         \
    do {                                                                                                \
        hipError_t _e = (expr);                                                                         \
        if (_e != hipSuccess) return bfail(b, DOPE_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

dope_status batch_run_iteration(dope_batch *b) {
    if (b->use_graph) {
        if (!b->graph_ready) {
            BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed), "graph capture begin");
            const hipError_t le = dope::launch_iteration(b->grp, b->stream);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(b->stream, &g);
            if (le != hipSuccess || ce != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bfail(b, DOPE_EDEVICE, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
            }
            b->graph = g;
            BHIP_TRY(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "graph instantiate");
            b->graph_ready = true;
        }
        BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream), "graph launch");
        return DOPE_OK;
    }
    BHIP_TRY(b, dope::launch_iteration(b->grp, b->stream), "iteration launch");
    return DOPE_OK;
}

dope_status batch_sync(dope_batch *b) {
    const size_t n = b->ctxs.size();
    BHIP_TRY(b, hipMemcpyAsync(b->hsum, b->dsum, n * 4 * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream),
             "summary readback");
    // poll the completion before blocking (see wait_stream)
    if (!b->ev_sync && hipEventCreateWithFlags(&b->ev_sync, hipEventDisableTiming) != hipSuccess) b->ev_sync = nullptr;
    bool done = false;
    if (b->ev_sync) {
        BHIP_TRY(b, hipEventRecord(b->ev_sync, b->stream), "event record");
        for (int spin = 0; spin <= 20000 && !done; ++spin) {
            const hipError_t q = hipEventQuery(b->ev_sync);
            if (q == hipSuccess) done = true;
            else if (q != hipErrorNotReady) return bfail(b, DOPE_EDEVICE, std::string("event query: ") + hipGetErrorString(q));
        }
    }
    if (!done) BHIP_TRY(b, hipStreamSynchronize(b->stream), "stream synchronize");
    for (dope_ctx *c : b->ctxs) c->dirty = true;
    return DOPE_OK;
}

dope_status batch_setup(dope_batch *b) {
    const size_t n = b->ctxs.size();
    BHIP_TRY(b, hipMemcpyAsync(b->dparams, b->hparams, n * 2 * sizeof(int32_t), hipMemcpyHostToDevice, b->stream),
             "parameter upload");
    BHIP_TRY(b, dope::launch_batch_setup(b->imgs, int32_t(n), b->dparams, b->stream), "batch setup launch");
    for (dope_ctx *c : b->ctxs) {
        c->validate_pending = false;   // taken by the batch setup kernel
        c->ctl_fresh = false;
    }
    return DOPE_OK;
}

// {t, halted, converged, status} of image i: the batch's summary when the batch ran the image last (its context
// is then marked dirty), otherwise the context's host mirror (the image was reset, set or read back since).
void image_summary(const dope_batch *b, size_t i, int32_t out[4]) {
    const dope_ctx *c = b->ctxs[i];
    if (c->dirty) {
        for (int f = 0; f < 4; ++f) out[f] = b->hsum[4 * i + f];
    } else {
        out[0] = c->hctl->t;
        out[1] = c->hctl->halted;
        out[2] = c->hctl->converged;
        out[3] = c->hctl->status;
    }
}

dope_status batch_status(dope_batch *b) {
    for (size_t i = 0; i < b->ctxs.size(); ++i)
        if (b->hsum[4 * i + 3] != 0)
            return bfail(b, dope_status(b->hsum[4 * i + 3]), "image " + std::to_string(i) + " stopped with an error");
    return DOPE_OK;
}

void batch_drop_graph(dope_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_ready = false;
}

// (Re)builds the batch's device arrays for ctxs, reusing its buffers when they are large enough.
dope_status batch_bind(dope_batch *b, dope_ctx *const *ctxs, int32_t n) {
    int conn = 0, solver = 0;
    for (int32_t i = 0; i < n; ++i) {
        dope_ctx *c = ctxs[i];
        if (!c) return bfail(b, DOPE_EINVAL, "null context");
        dope_status st = check_ready(c);
        if (st != DOPE_OK) return bfail(b, st, c->err);
        if (i == 0) { conn = c->g.conn; solver = c->solver; }
        if (c->g.conn != conn || c->solver != solver)
            return bfail(b, DOPE_EINVAL, "batch members must share connectivity and solver");
        if (c->gscr) return bfail(b, DOPE_EINVAL, "blocks beyond the LDS are solved one image at a time");
    }
    int64_t nblk = 0, nchk = 0, nrow = 0;
    int32_t npmax = 0;
    for (int32_t i = 0; i < n; ++i) {
        nblk += ctxs[i]->g.K;
        nchk += int64_t(ctxs[i]->hchunk.size());
        nrow += int64_t(ctxs[i]->g.H) * ctxs[i]->g.D;
        npmax = std::max(npmax, ctxs[i]->g.max_np);
    }
    if (nblk >= (int64_t(1) << 31) || nchk >= (int64_t(1) << 31) || nrow >= (int64_t(1) << 31))
        return bfail(b, DOPE_EINVAL, "batch too large");
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
    const size_t o_img = take(size_t(n) * sizeof(dope::Img)), o_bi = take(size_t(nblk) * sizeof(dope::Item)),
                 o_ci = take(size_t(nchk) * sizeof(dope::Item)), o_q = take(sizeof(dope::Queue)),
                 o_sum = take(size_t(n) * 16), o_par = take(size_t(n) * 8),
                 o_rows = take(size_t(nrow) * sizeof(dope::Item)), o_args = take(size_t(n) * sizeof(dope::SetupArg)),
                 o_labs = take(size_t(n) * sizeof(uint8_t *));
    if (o > b->dcap) {
        if (b->dbuf) (void)hipFree(b->dbuf);
        b->dbuf = nullptr;
        b->dcap = 0;
        void *ptr = nullptr;
        if (hipMalloc(&ptr, o + o / 2) != hipSuccess) {
            (void)hipGetLastError();
            return bfail(b, DOPE_ENOMEM, "batch buffer allocation failed");
        }
        b->dbuf = static_cast<char *>(ptr);
        b->dcap = o + o / 2;
    }
    if (size_t(n) > b->hcap) {
        if (b->ev_stage) (void)hipEventSynchronize(b->ev_stage);   // staging arrays may still be read
        if (b->hsum) (void)hipHostFree(b->hsum);
        if (b->hparams) (void)hipHostFree(b->hparams);
        if (b->hargs) (void)hipHostFree(b->hargs);
        if (b->hlabs) (void)hipHostFree(b->hlabs);
        b->hsum = b->hparams = nullptr;
        b->hargs = nullptr;
        b->hlabs = nullptr;
        b->hcap = 0;
        void *hs = nullptr, *hp = nullptr, *ha = nullptr, *hl = nullptr;
        const size_t cap = size_t(n) + size_t(n) / 2;
        if (hipHostMalloc(&hs, cap * 16, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&hp, cap * 8, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&ha, cap * sizeof(dope::SetupArg), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&hl, cap * sizeof(uint8_t *), hipHostMallocDefault) != hipSuccess) {
            if (hs) (void)hipHostFree(hs);
            if (hp) (void)hipHostFree(hp);
            if (ha) (void)hipHostFree(ha);
            return bfail(b, DOPE_ENOMEM, "pinned host allocation failed");
        }
        b->hsum = static_cast<int32_t *>(hs);
        b->hparams = static_cast<int32_t *>(hp);
        b->hargs = static_cast<dope::SetupArg *>(ha);
        b->hlabs = static_cast<uint8_t **>(hl);
        b->hcap = cap;
    }
    b->ctxs.assign(ctxs, ctxs + n);
    b->imgs = reinterpret_cast<dope::Img *>(b->dbuf + o_img);
    auto *bi = reinterpret_cast<dope::Item *>(b->dbuf + o_bi);
    auto *ci = reinterpret_cast<dope::Item *>(b->dbuf + o_ci);
    auto *q = reinterpret_cast<dope::Queue *>(b->dbuf + o_q);
    b->dsum = reinterpret_cast<int32_t *>(b->dbuf + o_sum);
    b->dparams = reinterpret_cast<int32_t *>(b->dbuf + o_par);
    b->rows = reinterpret_cast<dope::Item *>(b->dbuf + o_rows);
    b->n_rows = int32_t(nrow);
    b->dargs = reinterpret_cast<dope::SetupArg *>(b->dbuf + o_args);
    b->dlabs = reinterpret_cast<uint8_t **>(b->dbuf + o_labs);
    std::vector<dope::Img> himg(static_cast<size_t>(n));
    std::vector<dope::Item> hbi, hci, hrow;
    hbi.reserve(size_t(nblk));
    hci.reserve(size_t(nchk));
    hrow.reserve(size_t(nrow));
    for (int32_t i = 0; i < n; ++i) {
        dope_ctx *c = ctxs[i];
        himg[size_t(i)] = host_img(c);
        himg[size_t(i)].summary = b->dsum + 4 * i;
        for (int32_t k = 0; k < c->g.K; ++k) hbi.push_back(dope::Item{i, k});
        for (size_t k = 0; k < c->hchunk.size(); ++k) hci.push_back(dope::Item{i, int32_t(k)});
        for (int32_t r = 0; r < c->g.H * c->g.D; ++r) hrow.push_back(dope::Item{i, r});
        b->hsum[4 * i + 0] = c->hctl->t;
        b->hsum[4 * i + 1] = c->hctl->halted;
        b->hsum[4 * i + 2] = c->hctl->converged;
        b->hsum[4 * i + 3] = c->hctl->status;
    }
    const dope::Queue hq{};
    BHIP_TRY(b, hipMemcpyAsync(b->imgs, himg.data(), himg.size() * sizeof(dope::Img), hipMemcpyHostToDevice, b->stream),
             "descriptor upload");
    BHIP_TRY(b, hipMemcpyAsync(bi, hbi.data(), hbi.size() * sizeof(dope::Item), hipMemcpyHostToDevice, b->stream),
             "item upload");
    BHIP_TRY(b, hipMemcpyAsync(b->rows, hrow.data(), hrow.size() * sizeof(dope::Item), hipMemcpyHostToDevice,
                               b->stream), "row item upload");
    if (!hci.empty())
        BHIP_TRY(b, hipMemcpyAsync(ci, hci.data(), hci.size() * sizeof(dope::Item), hipMemcpyHostToDevice, b->stream),
                 "item upload");
    BHIP_TRY(b, hipMemcpyAsync(q, &hq, sizeof(hq), hipMemcpyHostToDevice, b->stream), "queue upload");
    BHIP_TRY(b, hipMemcpyAsync(b->dsum, b->hsum, size_t(n) * 16, hipMemcpyHostToDevice, b->stream), "summary upload");
    BHIP_TRY(b, hipStreamSynchronize(b->stream), "stream synchronize");
    const int32_t workers = b->grp.n_workers;
    b->grp = dope::Group{b->imgs, n, bi, int32_t(nblk), ci, int32_t(nchk), q, conn, solver, npmax, workers};
    batch_drop_graph(b);
    return DOPE_OK;
}

}  // namespace

extern "C" {

dope_status dope_batch_create(dope_ctx *const *ctxs, int32_t n, dope_batch **out) {
    if (!ctxs || n <= 0 || !out) return DOPE_EINVAL;
    *out = nullptr;
    for (int32_t i = 0; i < n; ++i)
        if (!ctxs[i]) return DOPE_EINVAL;
    dope_batch *b = new (std::nothrow) dope_batch();
    if (!b) return DOPE_ENOMEM;
    b->stream = ctxs[0]->stream;
    const dope_status st = batch_bind(b, ctxs, n);
    if (st != DOPE_OK) {
        ctxs[0]->err = b->err;
        dope_batch_destroy(b);
        return st;
    }
    *out = b;
    return DOPE_OK;
}

dope_status dope_batch_set_energy_async(dope_batch *b, const int32_t *const *u, const int32_t *const *w,
                                        const int32_t *lambda_q8, int32_t mem_kind) {
    if (!b || !u || !w || !lambda_q8) return DOPE_EINVAL;
    if (mem_kind != DOPE_MEM_HOST && mem_kind != DOPE_MEM_DEVICE) return bfail(b, DOPE_EINVAL, "bad mem_kind");
    const size_t n = b->ctxs.size();
    for (size_t i = 0; i < n; ++i) {
        if (!u[i] || !w[i]) return bfail(b, DOPE_EINVAL, "null input of image " + std::to_string(i));
        if (lambda_q8[i] < 0) return bfail(b, DOPE_EINVAL, "lambda must be >= 0 (image " + std::to_string(i) + ")");
    }
    // the pinned argument staging may still be read by the previous upload
    if (b->ev_stage) BHIP_TRY(b, hipEventSynchronize(b->ev_stage), "event synchronize");
    for (size_t i = 0; i < n; ++i) {
        dope_ctx *c = b->ctxs[i];
        const Geom &g = c->g;
        const int32_t *u_src = u[i], *w_src = w[i];
        if (mem_kind == DOPE_MEM_HOST) {
            BHIP_TRY(b, hipMemcpyAsync(c->u, u[i], size_t(g.n) * 4, hipMemcpyHostToDevice, b->stream), "unary upload");
            BHIP_TRY(b, hipMemcpyAsync(c->w, w[i], size_t(g.n) * g.hs * 4, hipMemcpyHostToDevice, b->stream),
                     "weight upload");
            u_src = c->u;
            w_src = c->w;
        }
        b->hargs[i] = dope::SetupArg{u_src, w_src, c->p.mu0, uint64_t(c->p.eps_q16) * uint64_t(c->p.eps_q16),
                                     lambda_q8[i], c->p.mu_fact_num, c->p.mu_fact_den,
                                     int32_t(c->solver != DOPE_SOLVER_MAXFLOW ? 1 : 0)};
    }
    BHIP_TRY(b, hipMemcpyAsync(b->dargs, b->hargs, n * sizeof(dope::SetupArg), hipMemcpyHostToDevice, b->stream),
             "argument upload");
    if (!b->ev_stage && hipEventCreateWithFlags(&b->ev_stage, hipEventDisableTiming) != hipSuccess) b->ev_stage = nullptr;
    if (b->ev_stage) BHIP_TRY(b, hipEventRecord(b->ev_stage, b->stream), "event record");
    BHIP_TRY(b, dope::launch_setup_batch(b->grp.conn, b->imgs, b->dargs, b->rows, b->n_rows, b->stream),
             "batched setup launch");
    for (size_t i = 0; i < n; ++i) {
        dope_ctx *c = b->ctxs[i];
        // host mirror of the reset state (as dope_set_energy_async); validation is taken by the next batch call
        Ctl h{};
        h.M = c->p.mu0;
        h.eps2 = uint64_t(c->p.eps_q16) * uint64_t(c->p.eps_q16);
        h.mu_num = c->p.mu_fact_num;
        h.mu_den = c->p.mu_fact_den;
        *c->hctl = h;
        c->dirty = false;
        c->lam_q8 = lambda_q8[i];
        c->energy_set = true;
        c->validate_pending = true;
        c->ctl_fresh = false;
        c->err.clear();
    }
    return DOPE_OK;
}

dope_status dope_batch_labels(dope_batch *b, uint8_t *const *labels, int32_t mem_kind) {
    if (!b || !labels) return DOPE_EINVAL;
    if (mem_kind != DOPE_MEM_HOST && mem_kind != DOPE_MEM_DEVICE) return bfail(b, DOPE_EINVAL, "bad mem_kind");
    const size_t n = b->ctxs.size();
    for (size_t i = 0; i < n; ++i)
        if (!labels[i]) return bfail(b, DOPE_EINVAL, "null labels of image " + std::to_string(i));
    if (b->ev_stage) BHIP_TRY(b, hipEventSynchronize(b->ev_stage), "event synchronize");
    for (size_t i = 0; i < n; ++i) b->hlabs[i] = mem_kind == DOPE_MEM_DEVICE ? labels[i] : b->ctxs[i]->labels;
    BHIP_TRY(b, hipMemcpyAsync(b->dlabs, b->hlabs, n * sizeof(uint8_t *), hipMemcpyHostToDevice, b->stream),
             "label pointer upload");
    if (!b->ev_stage && hipEventCreateWithFlags(&b->ev_stage, hipEventDisableTiming) != hipSuccess) b->ev_stage = nullptr;
    if (b->ev_stage) BHIP_TRY(b, hipEventRecord(b->ev_stage, b->stream), "event record");
    BHIP_TRY(b, dope::launch_labels_batch(b->imgs, b->dlabs, b->rows, b->n_rows, b->stream), "batched labels launch");
    if (mem_kind == DOPE_MEM_DEVICE) return DOPE_OK;   // stream-ordered, no wait
    for (size_t i = 0; i < n; ++i)
        BHIP_TRY(b, hipMemcpyAsync(labels[i], b->ctxs[i]->labels, size_t(b->ctxs[i]->g.n), hipMemcpyDeviceToHost,
                                   b->stream), "labels copy");
    BHIP_TRY(b, hipStreamSynchronize(b->stream), "stream synchronize");
    return DOPE_OK;
}

dope_status dope_batch_iterate(dope_batch *b, int32_t n_iter) {
    if (!b || n_iter < 0) return DOPE_EINVAL;
    const size_t n = b->ctxs.size();
    for (size_t i = 0; i < n; ++i) {
        int32_t sm[4];
        image_summary(b, i, sm);
        b->hparams[2 * i] = sm[0] + n_iter;
        b->hparams[2 * i + 1] = 0;
    }
    dope_status st = batch_setup(b);
    if (st != DOPE_OK) return st;
    for (int32_t it = 0; it < n_iter; ++it) {
        st = batch_run_iteration(b);
        if (st != DOPE_OK) return st;
    }
    st = batch_sync(b);
    if (st != DOPE_OK) return st;
    return batch_status(b);
}

dope_status dope_batch_solve(dope_batch *b) {
    if (!b) return DOPE_EINVAL;
    const size_t n = b->ctxs.size();
    int32_t most = 0;
    for (size_t i = 0; i < n; ++i) {
        const dope_ctx *c = b->ctxs[i];
        int32_t sm[4];
        image_summary(b, i, sm);
        const bool done = sm[3] != 0 || (sm[0] > 0 && sm[2]);
        b->hparams[2 * i] = done ? sm[0] : c->p.max_iter;   // finished images take no more iterations
        b->hparams[2 * i + 1] = 1;
        most = std::max(most, c->p.max_iter);
    }
    dope_status st = batch_setup(b);
    if (st != DOPE_OK) return st;
    // Iterations go out in chunks of 2, 2, 4, 8, ... with one summary readback per chunk; an image whose
    // stopping rule held, or that reached its limit, skips the rest of the chunk on the device.
    int32_t issued = 0, chunk = 2, n_chunks = 0;
    while (issued < most) {
        const int32_t count = std::min(chunk, most - issued);
        for (int32_t it = 0; it < count; ++it) {
            st = batch_run_iteration(b);
            if (st != DOPE_OK) return st;
        }
        issued += count;
        st = batch_sync(b);
        if (st != DOPE_OK) return st;
        bool running = false;
        for (size_t i = 0; i < n && !running; ++i)
            running = !b->hsum[4 * i + 1] && b->hsum[4 * i] < b->hparams[2 * i];
        if (!running) break;
        if (++n_chunks >= 2) chunk = std::min(2 * chunk, 64);
    }
    return batch_status(b);
}

dope_status dope_batch_set_graph(dope_batch *b, int32_t on) {
    if (!b) return DOPE_EINVAL;
    b->use_graph = on != 0;
    return DOPE_OK;
}

dope_status dope_batch_set_workers(dope_batch *b, int32_t nw) {
    if (!b || nw < 0) return DOPE_EINVAL;
    b->grp.n_workers = nw;
    batch_drop_graph(b);   // the captured launch has the old grid
    return DOPE_OK;
}

dope_status dope_batch_info(dope_batch *b, dope_info *infos) {
    if (!b || !infos) return DOPE_EINVAL;
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
        dope_ctx *c = b->ctxs[i];
        c->dirty = false;
        dope_status st = sync_ctl(c);
        if (st != DOPE_OK) return st;
        fill_info(c, &infos[i]);
    }
    return DOPE_OK;
}

const char *dope_batch_last_error(const dope_batch *b) { return b ? b->err.c_str() : ""; }

void dope_batch_destroy(dope_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_sync) (void)hipEventDestroy(b->ev_sync);
    if (b->ev_stage) (void)hipEventDestroy(b->ev_stage);
    if (b->hargs) (void)hipHostFree(b->hargs);
    if (b->hlabs) (void)hipHostFree(b->hlabs);
    if (b->dbuf) (void)hipFree(b->dbuf);
    if (b->hsum) (void)hipHostFree(b->hsum);
    if (b->hparams) (void)hipHostFree(b->hparams);
    delete b;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------------------
// Serving: FIFO admission by HBM footprint into one arena, one batched iteration per tick
// ------------------------------------------------------------------------------------------------------------

namespace {

struct SrvReq {
    int64_t ticket = 0;
    dope_params p{};
    const int32_t *u = nullptr, *w = nullptr;
    int32_t lam = 0, mem = 0;
    uint8_t *lab = nullptr;
    int32_t lab_mem = 0;
    size_t bytes = 0, off = 0;
    dope_ctx *ctx = nullptr;
    dope_info info{};
    int32_t status = 0;
    bool finished = false;
};

}  // namespace

struct dope_server {
    size_t budget = 0;
    int32_t max_active = 0;
    int32_t iters = 1;   // batched iterations per step
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *arena = nullptr;
    std::map<size_t, size_t> free_blocks;   // offset -> size
    size_t in_use = 0;
    std::deque<SrvReq *> waiting;
    std::vector<SrvReq *> active;
    std::unordered_map<int64_t, std::unique_ptr<SrvReq>> reqs;
    dope_batch *batch = nullptr;
    bool dirty = true;
    int64_t next_ticket = 1;
    int32_t conn = 0;
    std::string err;
};

namespace {

dope_status sfail(dope_server *s, dope_status st, const std::string &msg) {
    if (s) s->err = msg;
    return st;
}

bool arena_alloc(dope_server *s, size_t bytes, size_t *off) {
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second < bytes) continue;
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        s->free_blocks.erase(it);
        if (rest) s->free_blocks[at] = rest;
        s->in_use += bytes;
        return true;
    }
    return false;
}

void arena_free(dope_server *s, size_t off, size_t bytes) {
    s->in_use -= bytes;
    auto it = s->free_blocks.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != s->free_blocks.end() && it->first + it->second == next->first) {
        it->second += next->second;
        s->free_blocks.erase(next);
    }
    if (it != s->free_blocks.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            s->free_blocks.erase(it);
        }
    }
}

// Retire one admitted request: labels, final info, context and arena space released.
void srv_retire(dope_server *s, SrvReq *r, int32_t status) {
    dope_ctx *c = r->ctx;
    if (status == 0) (void)dope_labels(c, r->lab, r->lab_mem);
    c->dirty = false;
    if (sync_ctl(c) == DOPE_OK) fill_info(c, &r->info);
    r->status = status;
    r->finished = true;
    dope_destroy(c);
    r->ctx = nullptr;
    arena_free(s, r->off, r->bytes);
}

}  // namespace

extern "C" {

dope_status dope_server_create(const dope_server_params *sp, dope_server **out) {
    if (!sp || !out || sp->hbm_budget == 0 || sp->max_active <= 0 || sp->iters_per_step < 0 ||
        sp->iters_per_step > 1024)
        return DOPE_EINVAL;
    *out = nullptr;
    dope_server *s = new (std::nothrow) dope_server();
    if (!s) return DOPE_ENOMEM;
    s->budget = sp->hbm_budget & ~size_t(255);
    s->max_active = sp->max_active;
    s->iters = sp->iters_per_step > 0 ? sp->iters_per_step : 1;
    if (sp->stream) {
        s->stream = static_cast<hipStream_t>(sp->stream);
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) { delete s; return DOPE_EDEVICE; }
        s->own_stream = true;
    }
    void *ptr = nullptr;
    if (hipMalloc(&ptr, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return DOPE_ENOMEM;
    }
    s->arena = static_cast<char *>(ptr);
    s->free_blocks[0] = s->budget;
    s->batch = new (std::nothrow) dope_batch();
    if (!s->batch) { dope_server_destroy(s); return DOPE_ENOMEM; }
    s->batch->stream = s->stream;
    *out = s;
    return DOPE_OK;
}

dope_status dope_server_submit(dope_server *s, const dope_params *p, const int32_t *u, const int32_t *w,
                               int32_t lambda_q8, int32_t mem_kind, uint8_t *labels_out, int32_t labels_mem_kind,
                               int64_t *ticket) {
    if (!s || !p || !u || !w || !labels_out || !ticket) return DOPE_EINVAL;
    dope_params q = *p;
    q.stream = s->stream;
    const size_t bytes = dope_workspace_bytes(&q);
    if (bytes == 0) return sfail(s, DOPE_EINVAL, "invalid request parameters");
    {
        Geom g;
        if (!make_geom(&q, g, nullptr).empty() || gmem_stride(g))
            return sfail(s, DOPE_EINVAL, "blocks beyond the LDS are solved one image at a time");
    }
    if (s->conn == 0) s->conn = q.connectivity;
    if (q.connectivity != s->conn) return sfail(s, DOPE_EINVAL, "requests of a server must share connectivity");
    const size_t need = align256(bytes);
    if (need > s->budget) return sfail(s, DOPE_EBUSY, "request workspace exceeds the HBM budget");
    auto r = std::make_unique<SrvReq>();
    r->ticket = s->next_ticket++;
    r->p = q;
    r->u = u;
    r->w = w;
    r->lam = lambda_q8;
    r->mem = mem_kind;
    r->lab = labels_out;
    r->lab_mem = labels_mem_kind;
    r->bytes = need;
    *ticket = r->ticket;
    s->waiting.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
    return DOPE_OK;
}

dope_status dope_server_step(dope_server *s, int64_t *finished, int32_t max_finished, int32_t *n_finished) {
    if (!s) return DOPE_EINVAL;
    int32_t nf = 0;
    auto report = [&](int64_t t) {
        if (finished && nf < max_finished) finished[nf] = t;
        ++nf;
    };
    // admission: arrival order while the arena and the slot count allow
    while (!s->waiting.empty() && int32_t(s->active.size()) < s->max_active) {
        SrvReq *r = s->waiting.front();
        size_t off = 0;
        if (!arena_alloc(s, r->bytes, &off)) break;
        s->waiting.pop_front();
        dope_ctx *c = nullptr;
        dope_status st = dope_create(&r->p, &c);
        if (st == DOPE_OK) st = dope_bind_workspace(c, s->arena + off, r->bytes);
        if (st == DOPE_OK) st = dope_set_energy_async(c, r->u, r->w, r->lam, r->mem);
        if (st != DOPE_OK) {
            if (c) dope_destroy(c);
            arena_free(s, off, r->bytes);
            r->status = st;
            r->finished = true;
            report(r->ticket);
            continue;
        }
        r->ctx = c;
        r->off = off;
        s->active.push_back(r);
        s->dirty = true;
    }
    if (s->active.empty()) {
        if (n_finished) *n_finished = nf;
        return DOPE_OK;
    }
    dope_batch *b = s->batch;
    if (s->dirty) {
        std::vector<dope_ctx *> cs;
        cs.reserve(s->active.size());
        for (SrvReq *r : s->active) cs.push_back(r->ctx);
        dope_status st = batch_bind(b, cs.data(), int32_t(cs.size()));
        if (st != DOPE_OK) return sfail(s, st, b->err);
        for (size_t i = 0; i < cs.size(); ++i) {
            b->hparams[2 * i] = cs[i]->p.max_iter;
            b->hparams[2 * i + 1] = 1;
        }
        st = batch_setup(b);
        if (st != DOPE_OK) return sfail(s, st, b->err);
        s->dirty = false;
    }
    // the step's iterations back to back; requests that halt among them are skipped on the device
    dope_status st = DOPE_OK;
    for (int32_t it = 0; it < s->iters && st == DOPE_OK; ++it) st = batch_run_iteration(b);
    if (st == DOPE_OK) st = batch_sync(b);
    if (st != DOPE_OK) return sfail(s, st, b->err);
    // retire
    std::vector<SrvReq *> keep;
    keep.reserve(s->active.size());
    for (size_t i = 0; i < s->active.size(); ++i) {
        SrvReq *r = s->active[i];
        const int32_t t = b->hsum[4 * i], halted = b->hsum[4 * i + 1], status = b->hsum[4 * i + 3];
        if (halted || t >= r->p.max_iter) {
            srv_retire(s, r, status);
            report(r->ticket);
            s->dirty = true;
        } else {
            keep.push_back(r);
        }
    }
    s->active.swap(keep);
    if (n_finished) *n_finished = nf;
    return DOPE_OK;
}

dope_status dope_server_result(dope_server *s, int64_t ticket, dope_info *info, int32_t *status) {
    if (!s) return DOPE_EINVAL;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || !it->second->finished) return sfail(s, DOPE_EINVAL, "unknown or unfinished ticket");
    if (info) *info = it->second->info;
    if (status) *status = it->second->status;
    return DOPE_OK;
}

dope_status dope_server_load(const dope_server *s, int32_t *waiting, int32_t *active, size_t *hbm_in_use) {
    if (!s) return DOPE_EINVAL;
    if (waiting) *waiting = int32_t(s->waiting.size());
    if (active) *active = int32_t(s->active.size());
    if (hbm_in_use) *hbm_in_use = s->in_use;
    return DOPE_OK;
}

const char *dope_server_last_error(const dope_server *s) { return s ? s->err.c_str() : ""; }

void dope_server_destroy(dope_server *s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (SrvReq *r : s->active)
        if (r->ctx) dope_destroy(r->ctx);
    if (s->batch) dope_batch_destroy(s->batch);
    if (s->arena) (void)hipFree(s->arena);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------------------
// One whole solve in caller-provided device memory, for the entry point that allocates nothing
// ------------------------------------------------------------------------------------------------------------

namespace dope {

// dope_set_energy_async + dope_solve + dope_labels on a transient host-side context whose workspace is ws (device
// memory of at least the workspace size of p, 256-byte aligned).  Creates no stream, event, pinned buffer or
// device allocation: the loop control is copied back into host memory of the context and the stream synchronised
// at every readback.  u, w, labels are device pointers; the labels are complete on return.  Errors are reported
// through the thread's dope_last_error(NULL) message.
dope_status solve_in_buffer(const dope_params *p, void *ws, size_t bytes, const int32_t *u, const int32_t *w,
                            int32_t lambda_q8, uint8_t *labels, dope_info *out) {
    if (!p || !u || !w || !labels) {
        g_create_error = "null params, input or output";
        return DOPE_EINVAL;
    }
    dope_params q = *p;
    if (q.mu_fact_num == 0 && q.mu_fact_den == 0) { q.mu_fact_num = 21; q.mu_fact_den = 20; }
    dope_ctx c;
    std::vector<int32_t> bt;
    std::string msg = make_geom(&q, c.g, &bt);
    if (!msg.empty()) {
        g_create_error = msg;
        return DOPE_EINVAL;
    }
    const size_t need = layout_for(c.g).total;
    if (need > bytes) {
        g_create_error = "the problem needs " + std::to_string(need) + " bytes of device state, more than the " +
                         std::to_string(bytes) + " bytes of the static scratch buffer";
        return DOPE_EINVAL;
    }
    c.p = q;
    c.hbtab.swap(bt);
    if (!build_tables(c.g, c.hbtab, c.nbl, c.hchunk)) {
        g_create_error = "internal: boundary pixel table inconsistent with the partition";
        return DOPE_EINVAL;
    }
    c.stream = static_cast<hipStream_t>(q.stream);
    c.no_alloc = true;
    c.hctl = &c.hctl_host;
    c.ws = static_cast<char *>(ws);
    c.ws_bytes = bytes;
    c.own_ws = false;
    assign_pointers(&c);
    dope_status st = upload_tables(&c);
    if (st == DOPE_OK) st = dope_set_energy_async(&c, u, w, lambda_q8, DOPE_MEM_DEVICE);
    if (st == DOPE_OK) st = dope_solve(&c, out);
    if (st == DOPE_OK) st = dope_labels(&c, labels, DOPE_MEM_DEVICE);
    if (st == DOPE_OK && hipStreamSynchronize(c.stream) != hipSuccess) {
        (void)hipGetLastError();
        c.err = "stream synchronize after the labels";
        st = DOPE_EDEVICE;
    }
    g_create_error = st == DOPE_OK ? std::string() : c.err;
    return st;
}

}  // namespace dope
