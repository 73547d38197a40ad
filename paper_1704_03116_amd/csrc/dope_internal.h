// Internal declarations shared by the DOPE host runtime and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dope {

// One axis of the block partition: length N, block edge B, stride s = B - o, count nb.
// A single-block axis has B = s = N and nb = 1.  The reciprocals (of s, nb, B and the extent of the last block)
// let kernels divide by these with a double-precision estimate and an integer fix-up (see qdiv).
struct Axis {
    int32_t N, B, s, nb;
    double inv_s, inv_nb, inv_B, inv_last;
};

inline Axis make_axis(int32_t N, int32_t B, int32_t s, int32_t nb) {
    const int32_t last = N - (nb - 1) * s;
    return Axis{N, B, s, nb, 1.0 / s, 1.0 / nb, 1.0 / B, 1.0 / (last < B ? last : B)};
}

struct Geom {
    Axis ax[3];
    int32_t W, H, D;
    int32_t conn;       // 2D: 4, 8, 24 (5x5), 48 (7x7), 80 (9x9); 3D: 6, 32, 122, 256 (radius-2, -3, -4 balls)
    int32_t hs;         // half-stencil size
    int32_t rad;        // stencil radius: every neighbour offset lies in [-rad, rad] per axis
    int32_t K;          // number of blocks
    int32_t max_np;     // largest block size in pixels
    int64_t n;          // pixels
    int64_t tot;        // sum of block sizes
    int64_t span[3];    // sum of block extents along each axis
    int64_t n_interior; // block pixels interior to their block (see is_interior)
};

inline __host__ __device__ int32_t axis_ext(const Axis &a, int32_t t) {
    const int32_t e = a.N - t * a.s;
    return e < a.B ? e : a.B;
}

// Workgroups of a launch are dispatched to the XCDs round-robin (workgroup b runs on XCD b % 8) and every XCD
// has its own L2.  Workgroup b takes item xcd_item(b, n): XCD j gets the contiguous item range starting at
// j * (n / 8) + min(j, n % 8), so neighbouring blocks or chunks, which read the same halo lines, share an L2
// instead of fetching those lines once per XCD.  A bijection of [0, n).
constexpr int NUM_XCDS = 8;
inline __host__ __device__ int32_t xcd_item(int32_t b, int32_t n) {
    const int32_t j = b % NUM_XCDS, slot = b / NUM_XCDS;
    const int32_t base = n / NUM_XCDS, rem = n % NUM_XCDS;
    return j * base + (j < rem ? j : rem) + slot;
}

// Blocks of full extent B along an axis: all but a clipped last one.
inline __host__ __device__ int32_t axis_full(const Axis &a) { return a.nb - (axis_ext(a, a.nb - 1) < a.B ? 1 : 0); }

// Block solved by workgroup b of a one-image block-solve launch.  The blocks of full extent along every axis come
// first (raster order over their box), then every other block (raster order over the rest); within each of the
// two groups every XCD takes a contiguous range.  When the blocks outnumber the workgroups that fit the chip at
// once, a block's solve time grows with its pixel count, so the full blocks fill the first round and the clipped
// blocks of the far faces, half the size or less, the next; in raster order the clipped blocks are spread through
// both rounds.  A bijection of [0, K) (the context checks it when it is created).
inline __host__ __device__ int32_t block_at(const Geom &g, int32_t b) {
    const int32_t nbx = g.ax[0].nb, nby = g.ax[1].nb;
    const int32_t fx = axis_full(g.ax[0]), fy = axis_full(g.ax[1]), fz = axis_full(g.ax[2]);
    const int32_t nf = fx * fy * fz;
    if (b < nf) {
        const int32_t f = xcd_item(b, nf);
        const int32_t kx = f % fx, r = f / fx;
        return kx + nbx * (r % fy + nby * (r / fy));
    }
    int32_t r = xcd_item(b - nf, g.K - nf);
    const int32_t per_layer = nbx * nby - fx * fy;   // clipped blocks in each z layer below fz
    if (r < fz * per_layer) {
        const int32_t kz = r / per_layer;
        r -= kz * per_layer;
        const int32_t px = nbx - fx;   // clipped along x in each row below fy
        int32_t kx, ky;
        if (r < fy * px) {
            ky = r / px;
            kx = fx + (r - ky * px);
        } else {
            r -= fy * px;
            ky = fy + r / nbx;
            kx = r - (ky - fy) * nbx;
        }
        return kx + nbx * (ky + nby * kz);
    }
    return (r - fz * per_layer) + nbx * nby * fz;   // the z layers from fz on
}

// A pixel is interior to block (tx, ty, tz) when it and every pixel of its stencil box (offsets up to r per axis)
// lie in that block only.  Then both Hc terms of Eq. (10) vanish for it, S_m is its single copy, and no other
// block reads it.  Along one axis: lo <= x < hi with lo = start + o + r (0 for the first block),
// hi = end - o - r (N for the last block), o = B - s.
inline __host__ __device__ int32_t axis_interior_lo(const Axis &a, int32_t t, int32_t r) {
    return t > 0 ? t * a.s + (a.B - a.s) + r : 0;
}
inline __host__ __device__ int32_t axis_interior_hi(const Axis &a, int32_t t, int32_t r) {
    return t < a.nb - 1 ? t * a.s + axis_ext(a, t) - (a.B - a.s) - r : a.N;
}
inline __host__ __device__ bool axis_interior(const Axis &a, int32_t t, int32_t x, int32_t r) {
    return x >= axis_interior_lo(a, t, r) && x < axis_interior_hi(a, t, r);
}

// Start of block (tx, ty, tz) in the block-major vectors.  Blocks are ordered x-fastest and only the last block
// along an axis can be clipped, so the blocks before index t along an axis cover t * B pixels of that axis.
inline __host__ __device__ int64_t block_offset(const Geom &g, int32_t tx, int32_t ty, int32_t tz) {
    const int64_t Px = int64_t(tx) * g.ax[0].B, Py = int64_t(ty) * g.ax[1].B, Pz = int64_t(tz) * g.ax[2].B;
    const int64_t Ey = axis_ext(g.ax[1], ty), Ez = axis_ext(g.ax[2], tz);
    return Pz * g.span[1] * g.span[0] + Ez * (Py * g.span[0] + Ey * Px);
}

// Label slots per pixel (most blocks a pixel can lie in): 4 in 2D, 8 in 3D.
inline __host__ __device__ bool conn_is_3d(int32_t conn) { return conn == 6 || conn == 32 || conn == 122 || conn == 256; }
inline __host__ __device__ int slot_count(const Geom &g) { return conn_is_3d(g.conn) ? 8 : 4; }

inline __host__ __device__ bool is_interior(const Geom &g, int32_t tx, int32_t ty, int32_t tz, int32_t x, int32_t y,
                                            int32_t z) {
    return axis_interior(g.ax[0], tx, x, g.rad) && axis_interior(g.ax[1], ty, y, g.rad) &&
           axis_interior(g.ax[2], tz, z, g.rad);
}

// Device-resident loop control.  Written by the host only through k_ctl_* kernels or state uploads.
struct Ctl {
    int64_t M;                 // mu of the next iteration
    uint64_t max_resid;        // running max_k r_k of the iteration in flight
    uint64_t last_max_resid;   // max_k r_k of the last completed iteration
    uint64_t eps2;             // eps_q16^2
    int64_t energy;            // accumulator of the energy kernel
    int32_t t;                 // completed iterations
    int32_t t_limit;           // iterations with t >= t_limit are skipped
    int32_t stop_on_converge;  // dope_solve: halt when the stopping rule holds
    int32_t converged;
    int32_t halted;            // sticky stop: error, or converged under stop_on_converge
    int32_t status;            // 0 or a dope_status error code (sticky)
    int32_t ovf_pending;
    int32_t solver_err;
    uint32_t wg_counter;       // last-workgroup detection in the consensus kernel
    int32_t mu_num, mu_den;
    int32_t flags;             // set_energy validation bits being accumulated (see FLAG_*); cleared by validation
    int32_t vflags;            // validation bits of the last set_energy
    int32_t vpending;          // a set_energy awaits its validation (done by the next control setup kernel)
    int32_t allow_negative;    // the resolved solver of that set_energy accepts negative weights
    int32_t spare;
    int64_t seq;               // host mirror only: number of the readback whose loop-control kernel wrote it last
};

enum : int32_t { FLAG_OFFGRID = 1, FLAG_NEGATIVE = 2, FLAG_TOOBIG = 4 };

constexpr int32_t Y_ONE = 1 << 16;
constexpr int32_t Y_HALF = 1 << 15;
constexpr int64_t STATE_LIMIT = 1 << 22;
constexpr int64_t MU_MAX = (1 << 24) - 1;
constexpr int64_t CAP_SUM_LIMIT = int64_t(1) << 29;
constexpr int BTAB_STRIDE = 8;     // x0, y0, z0, ex, ey, ez, offset, pad

// Bytes of the per-node mask of live in-block directions (one bit per full-stencil direction).
inline __host__ __device__ constexpr int dir_mask_bytes(int hs) {
    return 2 * hs <= 8 ? 1 : (2 * hs <= 32 ? 4 : (2 * hs <= 64 ? 8 : (2 * hs <= 128 ? 16 : 32)));
}

// LDS bytes of the max-flow block kernel for a block of np pixels and half-stencil size hs: a 64-byte header,
// capacity and flow per half-edge, unary/excess, height, free list, direction mask (aligned to its size) and
// state bits per node.
inline __host__ __device__ constexpr size_t maxflow_lds_bytes(int np, int hs) {
    const int mb = dir_mask_bytes(hs);
    return 64 + size_t(np) * (8 * hs + 9 + mb) + (mb > 16 ? 32 : (mb > 8 ? 16 : (mb > 1 ? 8 : 0)));
}
// The same layout without the per-edge arrays (capacities and flows, 8h bytes per node): the LDS part of the
// global-memory block solver, whose edge arrays stay in global memory.
inline __host__ __device__ constexpr size_t maxflow_node_lds_bytes(int np, int hs) {
    return maxflow_lds_bytes(np, hs) - size_t(np) * 8 * hs;
}
constexpr size_t LDS_LIMIT = 163840;   // gfx950: 160 KiB per workgroup
// Dynamic LDS the max-flow block kernels may take: the rest of the 160 KiB holds their static arrays (the per-axis
// cover rows of a block).
constexpr size_t MAXFLOW_LDS_LIMIT = LDS_LIMIT - 1024;
// LDS bytes of the LSA-TR block kernel (stencils with one-byte direction masks: 4, 8 and 6 neighbours): the
// max-flow state, then per node the signed capacities of its half-edges, the clamped Eq. (8) unary, the mask of
// its in-block edges and its current label.
inline __host__ __device__ constexpr size_t lsatr_lds_bytes(int np, int hs) {
    return ((maxflow_lds_bytes(np, hs) + 15) & ~size_t(15)) + size_t(np) * (4 * hs + 6);
}
constexpr int LSATR_THREADS = 256;
constexpr int LSATR_MAX_NP = 16 * LSATR_THREADS;   // the residual lane sums assume at most 16 pixels per thread
// Blocks beyond the LDS: workgroup size of the global-memory block solver (1024 threads for the 3x3 stencils, 256
// for the wide ones, whose solver needs more registers) and its largest block (at most 16 pixels per thread).
constexpr int gmem_threads(int conn) { return (conn == 4 || conn == 8 || conn == 6) ? 1024 : 256; }
constexpr int gmem_max_np(int conn) { return 16 * gmem_threads(conn); }
constexpr int NUM_CUS = 256;          // MI355X compute units


constexpr int CHUNK = 256;

// Everything a kernel needs to work on one image; an array of these lives in device memory so that one launch
// can serve many images.
struct Img {
    Geom g;
    const int32_t *u, *w, *cw, *btab;
    const int2 *blist;         // (block-major index, block) of the copies that are not interior to their block
    const int32_t *chunk_k0;   // block of the first entry of every CHUNK entries of blist
    int32_t *Y, *A0, *A1, *stats;
    uint8_t *yhat;
    // Block labels by pixel: slot_count(g) bytes per pixel; byte e + 2b + 4a of pixel (x, y, z) is the label of
    // its copy in block (tx - e, ty - b, tz - a), (tx, ty, tz) the highest block containing it along each axis.
    uint8_t *yslot;
    int64_t *resid;
    Ctl *ctl;
    int32_t *summary;   // optional: {t, halted, converged, status} written after every iteration
    // Covers of every coordinate of each axis for offsets -1, 0, +1 (axis 0 at [0, W), axis 1 at [W, W + H), axis
    // 2 at [W + H, W + H + D)): {top block index, codes}, codes holding per offset t (bits 4 (t + 1) ..): the number
    // of blocks containing the coordinate x + t (0 off the axis) and top(x + t) - top(x) + 1 (2 bits each).
    const int2 *axrow;
    int32_t n_chunks;
    int32_t n_blist;
};

struct Item {
    int32_t img, idx;   // image, and block (solve), 256-pixel chunk (consensus) or pixel row (setup, labels)
};

// Per-image arguments of a batched energy upload.
struct SetupArg {
    const int32_t *u_src, *w_src;   // inputs in device memory (the workspace staging copies for host inputs)
    int64_t mu0;
    uint64_t eps2;
    int32_t lam_q8, mu_num, mu_den, allow_negative;
};

// Device work queue of the persistent block-solve launch; reset by the finalize kernel of each iteration.
struct Queue {
    uint32_t next;
    uint32_t pad[63];
};

// Device arrays describing one launch group (all images share connectivity and solver).
struct Group {
    const Img *imgs;
    int32_t n_imgs;
    const Item *blk_items;
    int32_t n_blk_items;
    const Item *chk_items;
    int32_t n_chk_items;
    Queue *queue;
    int32_t conn, solver, npmax;
    int32_t n_workers;   // workgroups of the persistent block-solve launch (0 = one per item)
    // One-image groups: host copy of the image descriptor, passed to the kernels by value, and the multiplier
    // buffer parity (t & 1) of the iteration being enqueued.  Null for batches (read from device memory).
    const Img *one = nullptr;
    int32_t par = 0;
    // One-image groups whose blocks exceed the LDS: the max-flow state of workgroup b lives at
    // gscratch + b * gstride (gstride >= maxflow_lds_bytes(npmax, h)); null otherwise.
    unsigned char *gscratch = nullptr;
    uint64_t gstride = 0;
};

// One ADMM iteration (block solves, consensus and multipliers, loop control) for every image of the group.
// mirror: host-visible copy of the one-image loop control that the finalize kernel refreshes (or nullptr)
// seq: written into the mirror after the rest of it (system-scope fence between), so that the host can poll it
hipError_t launch_iteration(const Group &grp, hipStream_t s, Ctl *mirror = nullptr, int64_t seq = 0);
// Per-image loop setup of a batch: params[2 i] = t_limit, params[2 i + 1] = stop_on_converge.
hipError_t launch_batch_setup(const Img *imgs, int32_t n, const int32_t *params, hipStream_t s);
// Individual phases (used for per-kernel timing).
// With events, the launch records its own dispatch start and end in e0 / e1 (hipExtLaunchKernel).
hipError_t launch_solve_phase(const Group &grp, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_consensus_phase(const Group &grp, hipStream_t s, hipEvent_t e0 = nullptr,
                                  hipEvent_t e1 = nullptr);
hipError_t launch_finalize_phase(const Group &grp, hipStream_t s, Ctl *mirror = nullptr, int64_t seq = 0);

// set_energy on the device: workspace copy of u (src != ws), c_ij, initial state and loop control, left as a
// solve with limit t_limit starts it.  The validation verdict (status / halted set on the device when the energy
// is invalid) is taken by the next launch_validate, launch_ctl_setup, launch_batch_setup or k_finalize; until
// then the iteration kernels skip an energy the verdict will reject.
hipError_t launch_validate(Ctl *ctl, hipStream_t s);
// Boundary list of one image (see the workspace layout): one workgroup per block writes the owner copies of the
// block's non-interior pixels from the block's base entry btab[k][7].
hipError_t launch_build_blist(const Geom &g, const int32_t *btab, int2 *blist, hipStream_t s);
// Axis cover rows of one image (see Img::axrow): W + H + D entries.
hipError_t launch_axis_rows(const Geom &g, int2 *axrow, hipStream_t s);
hipError_t launch_setup(const Geom &g, const int32_t *u_src, const int32_t *w_src, int32_t *u_ws, int32_t *cw,
                        int32_t lam_q8, int32_t *Y, int32_t *A0, int32_t *A1, uint8_t *yhat,
                        int64_t *resid, Ctl *ctl, int64_t mu0, int32_t mu_num, int32_t mu_den, uint64_t eps2,
                        int32_t allow_negative, int32_t t_limit, hipStream_t s);
hipError_t launch_ctl_setup(Ctl *ctl, int32_t t_limit, int32_t stop_on_converge, int32_t clear_energy,
                            hipStream_t s);
hipError_t launch_labels(const Geom &g, const int32_t *Y, uint8_t *labels, hipStream_t s);
// Batched energy upload and labels: one workgroup per (image, pixel row) item, n_rows items.
hipError_t launch_setup_batch(int32_t conn, const Img *imgs, const SetupArg *args, const Item *rows, int32_t n_rows,
                              hipStream_t s);
hipError_t launch_labels_batch(const Img *imgs, uint8_t *const *labels, const Item *rows, int32_t n_rows,
                               hipStream_t s);
// part: ENERGY_PARTS int64 of scratch.
hipError_t launch_energy(const Geom &g, const int32_t *u, const int32_t *cw, const int32_t *Y, int64_t *part,
                         Ctl *ctl, hipStream_t s);
constexpr int ENERGY_PARTS = 256;

}  // namespace dope
