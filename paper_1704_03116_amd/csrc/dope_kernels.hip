// gfx950 kernels of the DOPE ADMM iteration (Algorithm 1 of the paper).
//
//   k_setup             energy upload: copy of u, c_ij = lambda w 64 / (q_i q_j) with validation bits, initial
//                       state (Y = 1/2, A = 0) and loop control.
//   k_block_solve*      one workgroup per block: Eq. (8) unaries from Theorem 1's coupling terms, strictly forced
//                       nodes, forced-node elimination, push-relabel max preflow in LDS with breadth-first global
//                       relabels, canonical minimal cut -> yhat_k; Eq. (10)/(11) for the pixels interior to their
//                       block.  Variants: one image (descriptor as kernel argument, full blocks dispatched
//                       first), a batch (one workgroup per item), a batch over a persistent work queue, and one
//                       image with blocks beyond the LDS (edge arrays, or the whole state, in the workspace).
//   k_block_exhaustive  one wavefront per block of <= 16 pixels: Gray-code enumeration of all labellings,
//                       smallest-code minimiser (any sign of the pairwise weights).
//   k_block_lsatr       one workgroup per non-submodular block that fits the LDS: trust-region local submodular
//                       approximation steps, each a block max-flow of the linearised problem (3x3 stencils).
//   k_consensus*        one thread per boundary pixel: Eq. (10) consensus Y, Eq. (11) multipliers of its copies,
//                       per-block residual of the stopping rule.
//   k_finalize          loop control: max_k r_k, stopping rule, errors, mu and t.
//   k_labels, k_energy  labels [Y > 1/2] and the Eq. (1) energy.
//   k_build_blist       the consensus work list (owner copies of the pixels not interior to their block).
//   k_setup_batch, k_labels_batch, k_batch_setup, k_ctl_setup: the same set-up and outputs over a batch.
//
// Every kernel is a template over the stencil (CONN): 4- and 8-connected, 5x5, 7x7 and 9x9 squares in 2D;
// 6-connected and the radius-2, -3 and -4 balls in 3D.  All arithmetic is integer; every kernel checks the device loop control, so the
// host can enqueue several iterations ahead of the stopping rule without reading anything back.
#include "dope_internal.h"

#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>

// Loops over stencil directions are unrolled, except in the translation unit of the radius-4 ball (256
// neighbours), whose kernels keep them as loops: unrolled, that stencil's code would not fit the instruction cache
// nor build in reasonable time.
#if defined(DOPE_CONN) && DOPE_CONN == 256
#define DOPE_UNROLL _Pragma("nounroll")
#else
#define DOPE_UNROLL _Pragma("unroll")
#endif

namespace dope {

namespace {

// Pointers read from an image descriptor are generic (flat) to the compiler.  Cast to the global address space
// they give global loads and stores, which the scalar-load wait counter does not track, so gathers stay in flight
// across the scalar loads of descriptor fields instead of being drained before each of them.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T *gp(T *p) { return (GLOBAL T *)p; }

// Element at byte offset off of a global array: a uniform base plus a 32-bit lane offset, which the compiler
// issues as a load with the base in scalar registers and no 64-bit address arithmetic per lane.  Every array
// read this way is below 4 GiB: pixel and copy counts are below 2^30, and the label slots of a 3D grid (8 bytes
// per voxel) below 2^32 bytes.
template <class T>
__device__ __forceinline__ T ld_at(const GLOBAL T *base, uint32_t off) {
    return *reinterpret_cast<const GLOBAL T *>(reinterpret_cast<const GLOBAL char *>(base) + off);
}
template <class T>
__device__ __forceinline__ void st_at(GLOBAL T *base, uint32_t off, T v) {
    *reinterpret_cast<GLOBAL T *>(reinterpret_cast<GLOBAL char *>(base) + off) = v;
}

enum : uint8_t { ST_FIXED = 1, ST_LABEL = 2, ST_MARK = 8 };
constexpr int16_t H_INF = 0x7FFF;

// Stencils: H half-edges per pixel, radius R (every offset lies in [-R, R] per axis), grid dimension NDIM.
// CONN 24, 48 and 80 are the square 5x5, 7x7 and 9x9 neighbourhoods of a 2D grid, CONN 32 and 122 the radius-2
// and radius-3 balls of a 3D grid (the spherical kernels of size 5 and 7).
template <int CONN> struct Sten;
template <> struct Sten<4> { static constexpr int H = 2, R = 1, NDIM = 2; };
template <> struct Sten<8> { static constexpr int H = 4, R = 1, NDIM = 2; };
template <> struct Sten<24> { static constexpr int H = 12, R = 2, NDIM = 2; };
template <> struct Sten<48> { static constexpr int H = 24, R = 3, NDIM = 2; };
template <> struct Sten<80> { static constexpr int H = 40, R = 4, NDIM = 2; };
template <> struct Sten<6> { static constexpr int H = 3, R = 1, NDIM = 3; };
template <> struct Sten<32> { static constexpr int H = 16, R = 2, NDIM = 3; };
template <> struct Sten<122> { static constexpr int H = 61, R = 3, NDIM = 3; };
template <> struct Sten<256> { static constexpr int H = 128, R = 4, NDIM = 3; };

// Half-stencil of the radius-3 ball (the spherical kernel of size 7): offsets of length at most 3 whose first
// nonzero coordinate, from z down to x, is positive, ordered by z, then y, then x.
constexpr int8_t kBall3[61][3] = {
    {1, 0, 0}, {2, 0, 0}, {3, 0, 0}, {-2, 1, 0}, {-1, 1, 0}, {0, 1, 0}, {1, 1, 0}, {2, 1, 0}, {-2, 2, 0},
    {-1, 2, 0}, {0, 2, 0}, {1, 2, 0}, {2, 2, 0}, {0, 3, 0}, {-2, -2, 1}, {-1, -2, 1}, {0, -2, 1}, {1, -2, 1},
    {2, -2, 1}, {-2, -1, 1}, {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {2, -1, 1}, {-2, 0, 1}, {-1, 0, 1}, {0, 0, 1},
    {1, 0, 1}, {2, 0, 1}, {-2, 1, 1}, {-1, 1, 1}, {0, 1, 1}, {1, 1, 1}, {2, 1, 1}, {-2, 2, 1}, {-1, 2, 1},
    {0, 2, 1}, {1, 2, 1}, {2, 2, 1}, {-1, -2, 2}, {0, -2, 2}, {1, -2, 2}, {-2, -1, 2}, {-1, -1, 2}, {0, -1, 2},
    {1, -1, 2}, {2, -1, 2}, {-2, 0, 2}, {-1, 0, 2}, {0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {-2, 1, 2}, {-1, 1, 2},
    {0, 1, 2}, {1, 1, 2}, {2, 1, 2}, {-1, 2, 2}, {0, 2, 2}, {1, 2, 2}, {0, 0, 3}
};

// Half-stencil of the radius-4 ball (the spherical kernel of size 9): offsets of length at most 4 whose first
// nonzero coordinate, from z down to x, is positive, ordered by z, then y, then x.
constexpr int8_t kBall4[128][3] = {
    {1, 0, 0}, {2, 0, 0}, {3, 0, 0}, {4, 0, 0}, {-3, 1, 0}, {-2, 1, 0}, {-1, 1, 0}, {0, 1, 0}, {1, 1, 0}, {2, 1, 0},
    {3, 1, 0}, {-3, 2, 0}, {-2, 2, 0}, {-1, 2, 0}, {0, 2, 0}, {1, 2, 0}, {2, 2, 0}, {3, 2, 0}, {-2, 3, 0}, {-1, 3, 0},
    {0, 3, 0}, {1, 3, 0}, {2, 3, 0}, {0, 4, 0}, {-2, -3, 1}, {-1, -3, 1}, {0, -3, 1}, {1, -3, 1}, {2, -3, 1},
    {-3, -2, 1}, {-2, -2, 1}, {-1, -2, 1}, {0, -2, 1}, {1, -2, 1}, {2, -2, 1}, {3, -2, 1}, {-3, -1, 1}, {-2, -1, 1},
    {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {2, -1, 1}, {3, -1, 1}, {-3, 0, 1}, {-2, 0, 1}, {-1, 0, 1}, {0, 0, 1},
    {1, 0, 1}, {2, 0, 1}, {3, 0, 1}, {-3, 1, 1}, {-2, 1, 1}, {-1, 1, 1}, {0, 1, 1}, {1, 1, 1}, {2, 1, 1}, {3, 1, 1},
    {-3, 2, 1}, {-2, 2, 1}, {-1, 2, 1}, {0, 2, 1}, {1, 2, 1}, {2, 2, 1}, {3, 2, 1}, {-2, 3, 1}, {-1, 3, 1}, {0, 3, 1},
    {1, 3, 1}, {2, 3, 1}, {-1, -3, 2}, {0, -3, 2}, {1, -3, 2}, {-2, -2, 2}, {-1, -2, 2}, {0, -2, 2}, {1, -2, 2},
    {2, -2, 2}, {-3, -1, 2}, {-2, -1, 2}, {-1, -1, 2}, {0, -1, 2}, {1, -1, 2}, {2, -1, 2}, {3, -1, 2}, {-3, 0, 2},
    {-2, 0, 2}, {-1, 0, 2}, {0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {3, 0, 2}, {-3, 1, 2}, {-2, 1, 2}, {-1, 1, 2}, {0, 1, 2},
    {1, 1, 2}, {2, 1, 2}, {3, 1, 2}, {-2, 2, 2}, {-1, 2, 2}, {0, 2, 2}, {1, 2, 2}, {2, 2, 2}, {-1, 3, 2}, {0, 3, 2},
    {1, 3, 2}, {-1, -2, 3}, {0, -2, 3}, {1, -2, 3}, {-2, -1, 3}, {-1, -1, 3}, {0, -1, 3}, {1, -1, 3}, {2, -1, 3},
    {-2, 0, 3}, {-1, 0, 3}, {0, 0, 3}, {1, 0, 3}, {2, 0, 3}, {-2, 1, 3}, {-1, 1, 3}, {0, 1, 3}, {1, 1, 3}, {2, 1, 3},
    {-1, 2, 3}, {0, 2, 3}, {1, 2, 3}, {0, 0, 4}
};

// 256 direction bits (the radius-4 ball), with the operations the kernels apply to an integer mask: a bit test
// (m >> d) & 1, a single-bit set m |= Mask256(1) << d, and a test for no bit.
struct Mask256 {
    uint64_t w[4];
    Mask256() = default;
    __host__ __device__ constexpr Mask256(unsigned long long v) : w{v, 0, 0, 0} {}
    struct Bit {
        const Mask256 &m;
        int d;
        __device__ __forceinline__ uint32_t operator&(uint32_t v) const { return uint32_t(m.w[d >> 6] >> (d & 63)) & v; }
    };
    __device__ __forceinline__ Bit operator>>(int d) const { return Bit{*this, d}; }
    __device__ __forceinline__ Mask256 operator<<(int d) const {
        // only the one-bit mask is ever shifted
        Mask256 r(0ull);
        if (w[0] & 1ull) r.w[d >> 6] = 1ull << (d & 63);
        return r;
    }
    __device__ __forceinline__ Mask256 &operator|=(const Mask256 &o) {
        w[0] |= o.w[0]; w[1] |= o.w[1]; w[2] |= o.w[2]; w[3] |= o.w[3];
        return *this;
    }
    __device__ __forceinline__ bool operator!() const { return (w[0] | w[1] | w[2] | w[3]) == 0; }
};

// One bit per full-stencil direction.
template <int CONN>
using DirMask = typename std::conditional<
    (2 * Sten<CONN>::H <= 32), uint32_t,
    typename std::conditional<(2 * Sten<CONN>::H <= 64), uint64_t,
                              typename std::conditional<(2 * Sten<CONN>::H <= 128), unsigned __int128,
                                                        Mask256>::type>::type>::type;
// The per-node copy of that mask in LDS (see dir_mask_bytes).
template <int CONN>
using LdsMask = typename std::conditional<(2 * Sten<CONN>::H <= 8), uint8_t, DirMask<CONN>>::type;

// Half-stencil offsets (must match the weight layout of the public header).
template <int CONN>
__device__ __forceinline__ int3 half_off(int o) {
    if (CONN == 4) return o == 0 ? make_int3(1, 0, 0) : make_int3(0, 1, 0);
    if (CONN == 8) {
        switch (o) {
            case 0: return make_int3(1, 0, 0);
            case 1: return make_int3(0, 1, 0);
            case 2: return make_int3(1, 1, 0);
            default: return make_int3(-1, 1, 0);
        }
    }
    if (CONN == 24 || CONN == 48 || CONN == 80) {
        // (dx, 0) for dx = 1..R, then (dx, dy) for dy = 1..R and dx = -R..R (x fastest)
        constexpr int R = Sten<CONN>::R;
        if (o < R) return make_int3(o + 1, 0, 0);
        const int q = o - R;
        return make_int3(q % (2 * R + 1) - R, 1 + q / (2 * R + 1), 0);
    }
    if (CONN == 122) return make_int3(kBall3[o][0], kBall3[o][1], kBall3[o][2]);
    if (CONN == 256) return make_int3(kBall4[o][0], kBall4[o][1], kBall4[o][2]);
    if (CONN == 32) {
        // offsets of length at most 2 whose first nonzero coordinate, from z down to x, is positive; ordered by
        // z, then y, then x
        switch (o) {
            case 0: return make_int3(1, 0, 0);
            case 1: return make_int3(2, 0, 0);
            case 2: return make_int3(-1, 1, 0);
            case 3: return make_int3(0, 1, 0);
            case 4: return make_int3(1, 1, 0);
            case 5: return make_int3(0, 2, 0);
            case 6: return make_int3(-1, -1, 1);
            case 7: return make_int3(0, -1, 1);
            case 8: return make_int3(1, -1, 1);
            case 9: return make_int3(-1, 0, 1);
            case 10: return make_int3(0, 0, 1);
            case 11: return make_int3(1, 0, 1);
            case 12: return make_int3(-1, 1, 1);
            case 13: return make_int3(0, 1, 1);
            case 14: return make_int3(1, 1, 1);
            default: return make_int3(0, 0, 2);
        }
    }
    switch (o) {
        case 0: return make_int3(1, 0, 0);
        case 1: return make_int3(0, 1, 0);
        default: return make_int3(0, 0, 1);
    }
}

// Full stencil: d < H is +half_off(d), d >= H is -half_off(d - H).
template <int CONN>
__device__ __forceinline__ int3 full_dir(int d) {
    constexpr int H = Sten<CONN>::H;
    int3 v = half_off<CONN>(d < H ? d : d - H);
    if (d >= H) { v.x = -v.x; v.y = -v.y; v.z = -v.z; }
    return v;
}

// Block intervals containing coordinate x of one axis: t_hi and, when cnt == 2, also t_hi - 1.  Coordinates
// outside the axis return cnt = 0.
struct AxCov {
    int thi, cnt;
};

// q = floor(n / d) and rem = n - q d for 0 <= n < 2^31 and d >= 1, given inv = 1.0 / d: the double-precision
// estimate n * inv is within 2^-21 of n / d, so its truncation is q or q - 1 (q + 1 only in the limit) and one
// integer fix-up makes it exact.  About ten instructions against some forty for an integer division.
__device__ __forceinline__ int qdiv(int n, int d, double inv, int &rem) {
    int q = int(double(n) * inv);
    int r = n - q * d;
    const bool lo = r < 0, hi = r >= d;   // selects, not branches
    q += (hi ? 1 : 0) - (lo ? 1 : 0);
    r += lo ? d : (hi ? -d : 0);
    rem = r;
    return q;
}

// Reciprocal of the extent of block t along an axis (only the last block can be clipped).
__device__ __forceinline__ double axis_inv_ext(const Axis &a, int t) { return t == a.nb - 1 ? a.inv_last : a.inv_B; }

// Local coordinates of position p of a block with extents ex, ey (x fastest).
__device__ __forceinline__ int3 block_local(int p, int ex, int ey, double inv_ex, double inv_ey) {
    int lx, ly;
    const int r = qdiv(p, ex, inv_ex, lx);
    const int lz = qdiv(r, ey, inv_ey, ly);
    return make_int3(lx, ly, lz);
}

// Local coordinates of positions p0, p0 + stride, p0 + 2 stride, ... of a block with extents ex, ey (x fastest):
// the first from one division, the others by adding the stride in the block's mixed radix (one carry per axis at
// most, since each digit of the stride is below the extent).
struct LocalWalk {
    int lx, ly, lz, dx, dy, dz, ex, ey;
    __device__ __forceinline__ void init(int p0, int stride, int ex_, int ey_, double inv_ex, double inv_ey) {
        ex = ex_;
        ey = ey_;
        const int3 l = block_local(p0, ex, ey, inv_ex, inv_ey);
        const int3 d = block_local(stride, ex, ey, inv_ex, inv_ey);
        lx = l.x; ly = l.y; lz = l.z;
        dx = d.x; dy = d.y; dz = d.z;
    }
    __device__ __forceinline__ void next() {
        lx += dx;
        const int cx = lx >= ex ? 1 : 0;
        lx -= cx ? ex : 0;
        ly += dy + cx;
        const int cy = ly >= ey ? 1 : 0;
        ly -= cy ? ey : 0;
        lz += dz + cy;
    }
};

// Covers of x - R .. x + R (0 <= x < N, R at most the stride s when the axis has several blocks) from one
// division: floor((x + t) / s) differs from floor(x / s) by at most one, downwards when rem + t < 0 and upwards
// when rem + t >= s.
template <int R>
__device__ __forceinline__ void axis_cov(const Axis &a, int x, AxCov c[2 * R + 1]) {
    int rem;
    const int tr = qdiv(x, a.s, a.inv_s, rem);
    // t_hi of x is tm = min(tr, nb - 1); a neighbour's is one less or one more only when tr is not clamped.  The
    // start of block t_hi - 1, (t_hi - 1) s, follows from one product.
    const int tm = tr < a.nb - 1 ? tr : a.nb - 1;
    const int pm = (tm - 1) * a.s;
DOPE_UNROLL
    for (int t = 0; t <= 2 * R; ++t) {
        const int xx = x + t - R, d = rem + t - R;
        const bool dn = d < 0 && tr <= a.nb - 1, up = d >= a.s && tr < a.nb - 1;
        const int th = tm - (dn ? 1 : 0) + (up ? 1 : 0);
        const int ps = pm - (dn ? a.s : 0) + (up ? a.s : 0);
        const int two = (th >= 1 && xx < ps + a.B) ? 1 : 0;
        c[t] = (xx < 0 || xx >= a.N) ? AxCov{0, 0} : AxCov{th, 1 + two};
    }
}

// Covers of one pixel's stencil box along the three axes (the z axis of a 2D grid is a single layer).
template <int CONN>
struct BoxCov {
    static constexpr int R = Sten<CONN>::R;
    AxCov x[2 * R + 1], y[2 * R + 1], z[2 * R + 1];
    __device__ __forceinline__ void init(const Geom &g, int gx, int gy, int gz) {
        axis_cov<R>(g.ax[0], gx, x);
        axis_cov<R>(g.ax[1], gy, y);
        if (Sten<CONN>::NDIM == 3) {
            axis_cov<R>(g.ax[2], gz, z);
        } else {
DOPE_UNROLL
            for (int t = 0; t <= 2 * R; ++t) z[t] = AxCov{0, t == R ? 1 : 0};
        }
    }
    // The same covers from the image's axis rows (stencils of radius 1): three loads instead of three divisions.
    __device__ __forceinline__ void init_rows(const GLOBAL uint64_t *rows, const Geom &g, int gx, int gy, int gz) {
        static_assert(R == 1, "axis rows hold offsets -1, 0, +1");
        const uint64_t rx = rows[gx], ry = rows[g.W + gy], rz = rows[g.W + g.H + gz];
        unpack_row(rx, x);
        unpack_row(ry, y);
        unpack_row(rz, z);
    }
    // a row is the int2 {top block, codes}: the top block in the low 32 bits
    __device__ __forceinline__ static void unpack_row(uint64_t r, AxCov c[3]) {
        const int top = int(uint32_t(r)), codes = int(uint32_t(r >> 32));
DOPE_UNROLL
        for (int t = 0; t < 3; ++t) {
            const int code = (codes >> (4 * t)) & 15;
            c[t] = AxCov{top + ((code >> 2) & 3) - 1, code & 3};
        }
    }
    // cover of the pixel itself (offset 0) and of neighbour offset v along each axis
    __device__ __forceinline__ const AxCov &cx(int dx) const { return x[dx + R]; }
    __device__ __forceinline__ const AxCov &cy(int dy) const { return y[dy + R]; }
    __device__ __forceinline__ const AxCov &cz(int dz) const { return z[dz + R]; }
    // log2 q of the pixel at offset v (every cover count is 1 or 2 on the grid; an off-grid offset gives 0)
    __device__ __forceinline__ int lq(int3 v) const {
        return max(cx(v.x).cnt - 1, 0) + max(cy(v.y).cnt - 1, 0) + max(cz(v.z).cnt - 1, 0);
    }
};

// Label slot of the copy at local position (lx, ly, lz) of block (tx, ty, tz): e + 2b + 4a where e = 1 when the
// pixel also lies in block tx + 1 (local x >= s and a next block exists), i.e. the copy is in block top_x - 1.
__device__ __forceinline__ int label_slot(const Geom &g, int tx, int ty, int tz, int lx, int ly, int lz) {
    const int e = (lx >= g.ax[0].s && tx < g.ax[0].nb - 1) ? 1 : 0;
    const int b = (ly >= g.ax[1].s && ty < g.ax[1].nb - 1) ? 1 : 0;
    const int a = (lz >= g.ax[2].s && tz < g.ax[2].nb - 1) ? 1 : 0;
    return e + 2 * b + 4 * a;
}


__device__ __forceinline__ bool in_grid(const Geom &g, int x, int y, int z) {
    return x >= 0 && x < g.W && y >= 0 && y < g.H && z >= 0 && z < g.D;
}

__device__ __forceinline__ int64_t lin(const Geom &g, int x, int y, int z) {
    return int64_t(x) + int64_t(g.W) * (int64_t(y) + int64_t(g.H) * int64_t(z));
}


// Sum of x over the 64 lanes of a wavefront, returned in lane 63; every lane must be active.  Data-parallel
// primitive moves, no LDS: each lane adds its three predecessors in its row of 16, then rows add the partial sums
// of the preceding lanes 4 and 8 apart (upper banks only), then lane 15's total goes to row 1 and lane 31's to
// rows 2 and 3.
__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
    const int x0 = int(x);
    uint32_t v = x + uint32_t(__builtin_amdgcn_update_dpp(0, x0, 0x111, 0xf, 0xf, false)) +   // row_shr:1
                 uint32_t(__builtin_amdgcn_update_dpp(0, x0, 0x112, 0xf, 0xf, false)) +       // row_shr:2
                 uint32_t(__builtin_amdgcn_update_dpp(0, x0, 0x113, 0xf, 0xf, false));        // row_shr:3
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xf, 0xe, false));           // row_shr:4
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xf, 0xc, false));           // row_shr:8
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xa, 0xf, false));           // row_bcast:15
    v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xc, 0xf, false));           // row_bcast:31
    return v;
}

// 64-bit lane sum in lane 63, exact for lane values below 2^52: two 26-bit halves whose 64-lane sums fit 32 bits.
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
    const uint32_t lo = wave_sum32(uint32_t(x & ((1ull << 26) - 1)));
    const uint32_t hi = wave_sum32(uint32_t(x >> 26));
    return (static_cast<unsigned long long>(hi) << 26) + lo;
}

// Status an energy's validation bits give (FLAG_*): off-grid or oversized weights -> EINVAL (-1), a negative
// weight when the solver needs c_ij >= 0 -> ENOTSUBMODULAR (-4), else 0.
__device__ __forceinline__ int32_t energy_verdict(int32_t flags, int32_t allow_negative) {
    return (flags & (FLAG_OFFGRID | FLAG_TOOBIG)) ? -1 : (((flags & FLAG_NEGATIVE) && !allow_negative) ? -4 : 0);
}

// An iteration kernel does nothing once the loop halted or reached its limit, or while the verdict on the energy
// is pending and will reject it.
__device__ __forceinline__ bool ctl_skip(const Ctl *ctl) {
    const GLOBAL Ctl *c = gp(ctl);
    const int32_t halted = c->halted, t = c->t, t_limit = c->t_limit, vpending = c->vpending, flags = c->flags,
                  allow_negative = c->allow_negative;
    return halted != 0 || t >= t_limit || (vpending && energy_verdict(flags, allow_negative) != 0);
}

// floor(n / M) for M >= 1 and |n| < 2^53: a double-precision estimate within +-2 of the quotient, then an exact
// integer correction.
__device__ __forceinline__ int64_t floor_div_est(int64_t n, int64_t M, double invM) {
    int64_t q = int64_t(floor(double(n) * invM));
    int64_t r = n - q * M;
    while (r < 0) { --q; r += M; }
    while (r >= M) { ++q; r -= M; }
    return q;
}

// Bit d set when full-stencil neighbour d of (x, y, z) lies inside [0, X) x [0, Y) x [0, Z) (the grid, or a
// block in local coordinates).  The stencil is a compile-time constant, so this is 2R comparisons per axis.
template <int CONN>
__device__ __forceinline__ DirMask<CONN> inside_mask(int x, int y, int z, int X, int Y, int Z) {
    constexpr int R = Sten<CONN>::R;
    bool okx[2 * R + 1], oky[2 * R + 1], okz[2 * R + 1];
DOPE_UNROLL
    for (int t = -R; t <= R; ++t) {
        okx[t + R] = t < 0 ? x >= -t : (t > 0 ? x < X - t : true);
        oky[t + R] = t < 0 ? y >= -t : (t > 0 ? y < Y - t : true);
        okz[t + R] = t < 0 ? z >= -t : (t > 0 ? z < Z - t : true);
    }
    DirMask<CONN> m = 0;
DOPE_UNROLL
    for (int d = 0; d < 2 * Sten<CONN>::H; ++d) {
        const int3 v = full_dir<CONN>(d);
        const bool ok = okx[v.x + R] && oky[v.y + R] && okz[v.z + R];
        m |= ok ? (DirMask<CONN>(1) << d) : DirMask<CONN>(0);
    }
    return m;
}

// Global inputs of the Eq. (8) unary of one block pixel: u_i, Y_i, the pixel's multiplier, c_ij and Y_j of its
// full-stencil neighbours (bit d of ing: neighbour d is on the grid).
template <int CONN>
struct PixLoads {
    static constexpr int ND = 2 * Sten<CONN>::H;
    int32_t u, Y, a;
    int32_t cv[ND], yj[ND];
    DirMask<CONN> ing;
};

// Issues every load of PixLoads without waiting for any (an off-grid neighbour reads pixel i itself and is
// masked when the values are used).  Pixel and copy indices are below 2^30.
template <int CONN>
__device__ __forceinline__ void unary_loads(const Geom &g, const GLOBAL int32_t *__restrict__ u,
                                            const GLOBAL int32_t *__restrict__ cw,
                                            const GLOBAL int32_t *__restrict__ Y, const GLOBAL int32_t *__restrict__ A,
                                            uint32_t ci, int gx, int gy, int gz, PixLoads<CONN> &ld) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    const uint32_t i = uint32_t(gx) + uint32_t(g.W) * (uint32_t(gy) + uint32_t(g.H) * uint32_t(gz));
    const uint32_t bi = i << 2;
    ld.ing = inside_mask<CONN>(gx, gy, gz, g.W, g.H, g.D);
    ld.Y = ld_at(Y, bi);
    ld.a = ld_at(A, ci << 2);
DOPE_UNROLL
    for (int d = 0; d < ND; ++d) {
        const int3 v = full_dir<CONN>(d);
        const int32_t dl = v.x + g.W * (v.y + g.H * v.z);
        uint32_t bj = ((ld.ing >> d) & 1u) ? bi + (uint32_t(dl) << 2) : bi;
        asm("" : "+v"(bj));   // optimisation barrier only: keeps the loads unconditional
        const GLOBAL int32_t *cwo = cw + int64_t(d < H ? d : d - H) * g.n;
        ld.cv[d] = ld_at(cwo, d < H ? bi : bj);
        ld.yj[d] = ld_at(Y, bj);
    }
    // last: under register pressure the compiler reloads this base from the kernel arguments inside the pixel
    // loop, and the wait for that reload then holds back only this gather
    ld.u = ld_at(u, bi);
    // 3D (four voxels per thread, four wavefronts per SIMD): an optimisation barrier makes every value wait
    // until all loads are issued, so the compiler cannot wait for one gather before issuing the next (measured
    // 10 % faster there; in 2D, with two wavefronts per SIMD, the compiler's interleaving is faster)
    if constexpr (ND == 6) {
        asm("" : "+v"(ld.u), "+v"(ld.Y), "+v"(ld.a), "+v"(ld.cv[0]), "+v"(ld.cv[1]), "+v"(ld.cv[2]),
            "+v"(ld.cv[3]), "+v"(ld.cv[4]), "+v"(ld.cv[5]), "+v"(ld.yj[0]), "+v"(ld.yj[1]), "+v"(ld.yj[2]),
            "+v"(ld.yj[3]), "+v"(ld.yj[4]), "+v"(ld.yj[5]));
    }
}

// log2 q of a pixel's stencil box from per-axis bit rows: bit t + R of bx is log2 of the number of blocks that
// contain the x coordinate at offset t (0 off the grid), likewise by and bz.  A block builds the rows of its
// coordinates once (block_lq_rows), so its pixels skip the per-pixel cover computation of BoxCov.
template <int CONN>
struct TabCov {
    static constexpr int R = Sten<CONN>::R;
    uint32_t bx, by, bz;
    __device__ __forceinline__ int lq(int3 v) const {
        return int((bx >> (v.x + R)) & 1u) + int((by >> (v.y + R)) & 1u) + int((bz >> (v.z + R)) & 1u);
    }
};

// Per-axis rows of TabCov for the coordinates of one block (extents up to LQ_TAB per axis).
constexpr int LQ_TAB = 128;
template <int CONN, int NT>
__device__ __forceinline__ void block_lq_rows(const Geom &g, int x0, int y0, int z0, int ex, int ey, int ez,
                                              uint16_t (*rows)[LQ_TAB]) {
    constexpr int R = Sten<CONN>::R;
    for (int i = threadIdx.x; i < ex + ey + ez; i += NT) {
        const int a = i < ex ? 0 : (i < ex + ey ? 1 : 2);
        const int l = a == 0 ? i : (a == 1 ? i - ex : i - ex - ey);
        uint32_t bits = 0;
        if (a < Sten<CONN>::NDIM) {
            AxCov c[2 * R + 1];
            axis_cov<R>(g.ax[a], (a == 0 ? x0 : (a == 1 ? y0 : z0)) + l, c);
DOPE_UNROLL
            for (int t = 0; t <= 2 * R; ++t) bits |= uint32_t(c[t].cnt >= 2 ? 1 : 0) << t;
        }
        rows[a][l] = uint16_t(bits);
    }
}

// Eq. (8) unary of a block pixel (scaled by 2^14, unary floored) and its block-local edge data, from its loads and
// the covers of its stencil box (BoxCov or TabCov).  cap_out[o] = c for in-block half-edges (0 otherwise); mask
// bit d set for in-block neighbours with c != 0; sumc = sum of |c| over in-block neighbours.  q_j is a power of
// two: in 2D (q_j <= 4) F = (q_j - [j in k]) c fits 32 bits and each neighbour costs one 32 x 32 -> 64-bit
// multiply-add; in 3D (q_j <= 8) the other factor, (Y_i - Y_j)(q_j - [j in k]), fits 32 bits (|Y| <= 2^22) and
// multiplies c the same way.
template <int CONN, class Cov>
__device__ __forceinline__ int64_t unary_from_cov(const Cov &bc, const PixLoads<CONN> &ld, int64_t M, int lx,
                                                  int ly, int lz, int ex, int ey, int ez, int32_t *cap_out,
                                                  DirMask<CONN> &mask, int64_t &sumc) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    const int lqi = bc.lq(make_int3(0, 0, 0));
    const DirMask<CONN> inb_m = inside_mask<CONN>(lx, ly, lz, ex, ey, ez);   // in the block implies on the grid
    int64_t G = 0;
    int32_t sc = 0;   // sum of |c| < 2^29 (checked at upload)
    mask = 0;
DOPE_UNROLL
    for (int d = 0; d < ND; ++d) {
        const int3 v = full_dir<CONN>(d);
        const int32_t c = ((ld.ing >> d) & 1u) ? ld.cv[d] : 0;
        const bool inb = (inb_m >> d) & 1u;
        const int lqj = bc.lq(v);
        // x (2^lqj - [j in k]) as a shift and a subtraction (the shift on the unsigned bits: |x 2^lqj| < 2^31)
        if (Sten<CONN>::NDIM == 2) {
            const int32_t F = int32_t(uint32_t(c) << lqj) - (inb ? c : 0);
            G += int64_t(F) * int64_t(ld.Y - ld.yj[d]);
        } else {
            const int32_t dy = ld.Y - ld.yj[d];
            const int32_t t = int32_t(uint32_t(dy) << lqj) - (inb ? dy : 0);
            G += int64_t(c) * int64_t(t);
        }
        if (d < H) cap_out[d] = inb ? c : 0;
        const bool on = inb && c != 0;
        sc += on ? (c < 0 ? -c : c) : 0;
        mask |= on ? (DirMask<CONN>(1) << d) : DirMask<CONN>(0);
    }
    sumc = sc;
    const int64_t mu_term = (M << 14) * int64_t(ld.a - ld.Y + Y_HALF);
    return int64_t(ld.u) * int64_t(16384 >> lqi) + ((G + mu_term) >> 16);
}

// The same unary for the wide stencils, CH directions at a time: the gathers of one chunk are in flight together
// and a pixel never holds more than CH neighbours' values (PixLoads holds two per direction, which beyond a few
// dozen directions spills registers).  The capacities of the in-block half-edges go straight to cap[o * npmax].
template <int CONN, int CH, class Cov>
__device__ __forceinline__ int64_t unary_chunked(const Geom &g, const GLOBAL int32_t *__restrict__ u,
                                                 const GLOBAL int32_t *__restrict__ cw,
                                                 const GLOBAL int32_t *__restrict__ Y,
                                                 const GLOBAL int32_t *__restrict__ A, uint32_t ci, int gx, int gy,
                                                 int gz, const Cov &bc, int64_t M, int lx, int ly, int lz, int ex,
                                                 int ey, int ez, int32_t *cap, int npmax, DirMask<CONN> &mask,
                                                 int64_t &sumc) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    const uint32_t i = uint32_t(gx) + uint32_t(g.W) * (uint32_t(gy) + uint32_t(g.H) * uint32_t(gz));
    const uint32_t bi = i << 2;
    const DirMask<CONN> ing = inside_mask<CONN>(gx, gy, gz, g.W, g.H, g.D);
    const int32_t uu = ld_at(u, bi), Yi = ld_at(Y, bi), a = ld_at(A, ci << 2);
    const int lqi = bc.lq(make_int3(0, 0, 0));
    const DirMask<CONN> inb_m = inside_mask<CONN>(lx, ly, lz, ex, ey, ez);   // in the block implies on the grid
    int64_t G = 0;
    int32_t sc = 0;   // sum of |c| < 2^29 (checked at upload)
    mask = 0;
#pragma nounroll
    for (int d0 = 0; d0 < ND; d0 += CH) {
        int32_t cv[CH], yj[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            // slots past the last direction gather direction ND - 1 again (unused)
            const int d = d0 + j < ND ? d0 + j : ND - 1;
            const int3 v = full_dir<CONN>(d);
            const int32_t dl = v.x + g.W * (v.y + g.H * v.z);
            uint32_t bj = ((ing >> d) & 1u) ? bi + (uint32_t(dl) << 2) : bi;
            asm("" : "+v"(bj));   // optimisation barrier only: keeps the loads unconditional
            const GLOBAL int32_t *cwo = cw + int64_t(d < H ? d : d - H) * g.n;
            cv[j] = ld_at(cwo, d < H ? bi : bj);
            yj[j] = ld_at(Y, bj);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int d = d0 + j;
            if (d >= ND) break;
            const int3 v = full_dir<CONN>(d);
            const int32_t c = ((ing >> d) & 1u) ? cv[j] : 0;
            const bool inb = (inb_m >> d) & 1u;
            const int lqj = bc.lq(v);
            if (Sten<CONN>::NDIM == 2) {
                const int32_t F = int32_t(uint32_t(c) << lqj) - (inb ? c : 0);
                G += int64_t(F) * int64_t(Yi - yj[j]);
            } else {
                const int32_t dy = Yi - yj[j];
                const int32_t t = int32_t(uint32_t(dy) << lqj) - (inb ? dy : 0);
                G += int64_t(c) * int64_t(t);
            }
            if (d < H) cap[d * npmax] = inb ? c : 0;
            const bool on = inb && c != 0;
            sc += on ? (c < 0 ? -c : c) : 0;
            mask |= on ? (DirMask<CONN>(1) << d) : DirMask<CONN>(0);
        }
    }
    sumc = sc;
    const int64_t mu_term = (M << 14) * int64_t(a - Yi + Y_HALF);
    return int64_t(uu) * int64_t(16384 >> lqi) + ((G + mu_term) >> 16);
}

template <int CONN>
__device__ __forceinline__ int64_t unary_from(const Geom &g, const PixLoads<CONN> &ld, int64_t M, int gx, int gy,
                                              int gz, int lx, int ly, int lz, int ex, int ey, int ez,
                                              int32_t *cap_out, DirMask<CONN> &mask, int64_t &sumc) {
    BoxCov<CONN> bc;
    bc.init(g, gx, gy, gz);
    return unary_from_cov<CONN>(bc, ld, M, lx, ly, lz, ex, ey, ez, cap_out, mask, sumc);
}

// ------------------------------------------------------------------------------------------------------------
// Max-flow block solve
// ------------------------------------------------------------------------------------------------------------

// Synchronisation of one phase of the flow computation over the free-node list.  BlockSync: the whole
// workgroup takes part (barriers, one per OR-reduction thanks to three rotating flag slots in LDS).  WaveSync: a
// single wavefront does the work with wave-scope fences and ballots, so no workgroup barrier is paid per pass.
struct BlockSync {
    int idx, step;
    int *slots;
    int phase;
    __device__ __forceinline__ void sync() { __syncthreads(); }
    __device__ __forceinline__ bool any(bool f) {
        int *sl = slots + phase;
        if (f) *sl = 1;
        __syncthreads();
        const bool r = *sl != 0;
        if (threadIdx.x == 0) slots[(phase + 2) % 3] = 0;   // the slot of the call after next
        phase = (phase + 1) % 3;
        return r;
    }
    // OR of the two low bits of f over the workgroup (one barrier; one LDS atomic per wavefront)
    __device__ __forceinline__ int bits(int f) {
        int *sl = slots + phase;
        const int w = (__any(f & 1) ? 1 : 0) | (__any(f & 2) ? 2 : 0);
        if ((threadIdx.x & 63) == 0 && w) atomicOr(sl, w);
        __syncthreads();
        const int r = *sl;
        if (threadIdx.x == 0) slots[(phase + 2) % 3] = 0;   // the slot of the call after next
        phase = (phase + 1) % 3;
        return r;
    }
};

struct WaveSync {
    int idx, step;
    __device__ __forceinline__ void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ __forceinline__ bool any(bool f) {
        sync();
        return __any(f ? 1 : 0) != 0;
    }
    __device__ __forceinline__ int bits(int f) {
        sync();
        int r = f;
DOPE_UNROLL
        for (int s = 32; s >= 1; s >>= 1) r |= __shfl_xor(r, s);
        return r;
    }
};

// LDS-resident block graph (see maxflow_lds_bytes).
template <int CONN>
struct BlockLds {
    static constexpr int H = Sten<CONN>::H;
    int32_t *cap;      // [H][npmax] capacity of the half-edge p -> p + off_o (0 when absent)
    int32_t *flw;      // [H][npmax] flow on that half-edge
    int32_t *dd;       // unary during elimination, then excess minus sink residual
    int16_t *hh;       // heights
    int16_t *lst;      // free nodes after the prologue's forcing test
    LdsMask<CONN> *msk;   // live in-block directions
    uint8_t *st;       // ST_* bits
    int npmax;
    int loff[H];

    __device__ __forceinline__ int nbr(int p, int d) const { return d < H ? p + loff[d] : p - loff[d - H]; }
    __device__ __forceinline__ int32_t capd(int p, int d) const {
        return d < H ? cap[d * npmax + p] : cap[(d - H) * npmax + p - loff[d - H]];
    }
    // residual of the arc p -> nbr(p, d)
    __device__ __forceinline__ int32_t res(int p, int d) const {
        if (d < H) return cap[d * npmax + p] - flw[d * npmax + p];
        const int v = p - loff[d - H];
        return cap[(d - H) * npmax + v] + flw[(d - H) * npmax + v];
    }
    // residual of the arc nbr(p, d) -> p
    __device__ __forceinline__ int32_t res_in(int p, int d) const {
        if (d < H) return cap[d * npmax + p] + flw[d * npmax + p];
        const int v = p - loff[d - H];
        return cap[(d - H) * npmax + v] - flw[(d - H) * npmax + v];
    }
    __device__ __forceinline__ void push(int p, int d, int32_t delta) {
        if (d < H) flw[d * npmax + p] += delta;
        else flw[(d - H) * npmax + p - loff[d - H]] -= delta;
    }
};

struct FlowStats {
    int rounds, grel, casc;
    bool fail;
};

// Everything after the prologue for the nfree nodes of lst: elimination of the nodes that the reduced problem
// forces, push-relabel to a max preflow, and the canonical cut (ST_MARK = label 1).
// Forced-node elimination over the nfree nodes of lst; returns whether any node is left free.
template <int CONN, class Sync>
__device__ __forceinline__ bool eliminate(Sync &sy, BlockLds<CONN> &L, int nfree, FlowStats &fs) {
    constexpr int ND = 2 * Sten<CONN>::H;
    // (1) a node is forced when its unary, with the pairwise terms of its fixed neighbours folded in, exceeds the
    //     total capacity towards its free neighbours.  Forcing only grows as neighbours get fixed, so passes may
    //     see each other's updates in any order and still reach the same fixed point.
    //     Each wavefront repeats its share of the list until it stops changing before the workgroup-wide
    //     reduction, so chains of forcings inside a wavefront's share cost no barrier.
    //     Bit 0 of the reduction: a node got fixed in this pass; bit 1: a node was still free after its visit in
    //     the wavefront's last sweep.
    for (;;) {
        int ch = 0;
        for (;;) {
            int wch = 0;
            for (int i = sy.idx; i < nfree; i += sy.step) {
                const int p = L.lst[i];
                if (L.st[p] & ST_FIXED) continue;
                const DirMask<CONN> m = L.msk[p];
                int32_t U = L.dd[p], S = 0;
DOPE_UNROLL
                for (int d = 0; d < ND; ++d)
                    if ((m >> d) & 1u) {
                        const uint8_t sv = L.st[L.nbr(p, d)];
                        const int32_t c = L.capd(p, d);
                        if (sv & ST_FIXED) U += (sv & ST_LABEL) ? -c : c;
                        else S += c;
                    }
                if (U < -S) { L.st[p] = ST_FIXED | ST_LABEL; wch |= 1; }
                else if (U > S) { L.st[p] = ST_FIXED; wch |= 1; }
                else wch |= 2;
            }
            if (!__any(wch & 1)) {
                ch |= wch;     // this sweep's still-free bit is exact for the wavefront's share
                break;
            }
            ch |= wch & 1;
        }
        ++fs.casc;
        const int r = sy.bits(ch);
        if (!(r & 1)) {
            // a pass without changes: a node still free was seen free by this pass, so bit 1 is exact here
            return (r & 2) != 0;
        }
    }
}

// The same elimination with each thread's list entries (at most MAXPT of them), their unaries and their live
// capacities held in registers across sweeps: a sweep then reads only the state bytes of the neighbours, instead
// of the node's own state, mask, unary and capacities as well.  Nodes are fixed only by the thread that holds
// them, so a node a thread has fixed is simply dropped from its registers.
template <int CONN, class Sync, int MAXPT>
__device__ __forceinline__ bool eliminate_cached(Sync &sy, BlockLds<CONN> &L, int nfree, FlowStats &fs) {
    constexpr int ND = 2 * Sten<CONN>::H;
    int pn[MAXPT];
    int32_t ub[MAXPT];
    int32_t cb[MAXPT][ND];
DOPE_UNROLL
    for (int j = 0; j < MAXPT; ++j) {
        const int i = sy.idx + j * sy.step;
        pn[j] = -1;
        ub[j] = 0;
DOPE_UNROLL
        for (int d = 0; d < ND; ++d) cb[j][d] = 0;
        if (i < nfree) {
            const int p = L.lst[i];
            if (!(L.st[p] & ST_FIXED)) {
                const DirMask<CONN> m = L.msk[p];
                pn[j] = p;
                ub[j] = L.dd[p];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) cb[j][d] = ((m >> d) & 1u) ? L.capd(p, d) : 0;
            }
        }
    }
    for (;;) {
        int ch = 0;
        for (;;) {
            int wch = 0;
DOPE_UNROLL
            for (int j = 0; j < MAXPT; ++j) {
                const int p = pn[j];
                if (p < 0) continue;
                uint8_t sv[ND];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) sv[d] = L.st[cb[j][d] ? L.nbr(p, d) : p];   // dead directions read p
                int32_t U = ub[j], S = 0;
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) {
                    const int32_t c = cb[j][d];
                    if (sv[d] & ST_FIXED) U += (sv[d] & ST_LABEL) ? -c : c;   // c = 0 for dead directions
                    else S += c;
                }
                if (U < -S) { L.st[p] = ST_FIXED | ST_LABEL; pn[j] = -1; wch |= 1; }
                else if (U > S) { L.st[p] = ST_FIXED; pn[j] = -1; wch |= 1; }
                else wch |= 2;
            }
            if (!__any(wch & 1)) {
                ch |= wch;
                break;
            }
            ch |= wch & 1;
        }
        ++fs.casc;
        const int r = sy.bits(ch);
        if (!(r & 1)) return (r & 2) != 0;
    }
}

// The same elimination for lists longer than the registers hold, B list entries per thread at a time: the
// entries' state, masks, unaries, capacities and neighbour states are all loaded before any of them is tested,
// so the loads of a batch overlap (with the capacities in global memory, one round trip per batch instead of one
// per entry).  A test may then miss a neighbour fixed earlier in the same batch; a later sweep sees it, as it sees
// any other update, and the fixed point is the same.
// Only nodes with a neighbour fixed since their last test can change, so a node is tested again only when its
// flag in the height array (unused until the flow phases) is set: every listed node starts flagged, and fixing a
// node flags its in-block neighbours.  A flag set while its node is being tested may be lost; so a pass without
// changes is followed by one that tests every free node, and only a full pass without changes ends the loop.
template <int CONN, class Sync, int B>
__device__ __forceinline__ bool eliminate_batched(Sync &sy, BlockLds<CONN> &L, int nfree, FlowStats &fs) {
    constexpr int ND = 2 * Sten<CONN>::H;
    for (int i = sy.idx; i < nfree; i += sy.step) L.hh[L.lst[i]] = 1;
    sy.sync();
    bool full = false;
    for (;;) {
        int ch = 0;
        for (;;) {
            int wch = 0;
            for (int i0 = sy.idx; i0 < nfree; i0 += B * sy.step) {
                int pb[B];
                int32_t ub[B], cb[B][ND];
                uint8_t sv[B][ND];
                DirMask<CONN> mb[B];
DOPE_UNROLL
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + j * sy.step;
                    pb[j] = i < nfree ? int(L.lst[i]) : -1;
                }
DOPE_UNROLL
                for (int j = 0; j < B; ++j) {
                    const int p = pb[j];
                    const bool live = p >= 0 && !(L.st[p] & ST_FIXED) && (full || L.hh[p] != 0);
                    if (live) L.hh[p] = 0;
                    const DirMask<CONN> m = live ? DirMask<CONN>(L.msk[p]) : DirMask<CONN>(0);
                    mb[j] = m;
                    ub[j] = live ? L.dd[p] : 0;
                    if (!live) pb[j] = -1;
DOPE_UNROLL
                    for (int d = 0; d < ND; ++d) {
                        const bool on = (m >> d) & 1u;
                        cb[j][d] = on ? L.capd(p, d) : 0;
                        sv[j][d] = on ? L.st[L.nbr(p, d)] : uint8_t(0);
                    }
                }
DOPE_UNROLL
                for (int j = 0; j < B; ++j) {
                    const int p = pb[j];
                    if (p < 0) continue;
                    int32_t U = ub[j], S = 0;
DOPE_UNROLL
                    for (int d = 0; d < ND; ++d) {
                        const int32_t c = cb[j][d];
                        if (sv[j][d] & ST_FIXED) U += (sv[j][d] & ST_LABEL) ? -c : c;
                        else S += c;
                    }
                    uint8_t fx = 0;
                    if (U < -S) fx = ST_FIXED | ST_LABEL;
                    else if (U > S) fx = ST_FIXED;
                    if (fx) {
                        L.st[p] = fx;
                        wch |= 1;
DOPE_UNROLL
                        for (int d = 0; d < ND; ++d)
                            if ((mb[j] >> d) & 1u) L.hh[L.nbr(p, d)] = 1;
                    } else {
                        wch |= 2;
                    }
                }
            }
            if (!__any(wch & 1)) {
                ch |= wch;
                break;
            }
            ch |= wch & 1;
        }
        ++fs.casc;
        const int r = sy.bits(ch);
        if (r & 1) {
            full = false;
        } else {
            // bit 1 is exact only when the pass tested every free node
            if (full) return (r & 2) != 0;
            full = true;
        }
    }
}

// Elimination, with the register-held variant when every thread has at most MAXPT list entries and the stencil
// has at most eight directions.  MAXPT is fixed per kernel (registers are allocated for the whole kernel): 4 for
// 1024-thread workgroups (16^3 blocks), 2 for 512 (32x32), 1 for 256 and for a single wavefront.  Longer lists
// with such a stencil take the batched variant (B > 0 entries per thread at a time).
template <int CONN, int MAXPT, class Sync, int B = 0>
__device__ __forceinline__ bool eliminate_fast(Sync &sy, BlockLds<CONN> &L, int nfree, FlowStats &fs) {
    if constexpr (2 * Sten<CONN>::H <= 8) {
        if (nfree <= MAXPT * sy.step) return eliminate_cached<CONN, Sync, MAXPT>(sy, L, nfree, fs);
        if constexpr (B > 0) return eliminate_batched<CONN, Sync, B>(sy, L, nfree, fs);
    }
    return eliminate<CONN>(sy, L, nfree, fs);
}

template <int NT>
constexpr int elim_regs() { return NT >= 1024 ? 4 : (NT >= 512 ? 2 : 1); }

// Forced-node elimination over the nodes p0 <= p < p1 of a block only, for the workgroups of k_block_prep_gmem that
// share a block: the neighbours outside the slice count as free (their capacities and states belong to another
// workgroup).  That only weakens the test -- a fixed neighbour moves its capacity from the free total into the
// unary -- so every node fixed here is fixed by the whole block's elimination as well, which then starts from
// these states and reaches the same fixed point.  s_lst / s_sum: the slice's list (nf entries, at most MAXPT per
// thread) and each entry's total in-block capacity; s_st: the slice's states (index p - p0).  The entries, their
// unaries and the capacities towards the slice are held in registers across sweeps, as in eliminate_cached.
template <int CONN, int MAXPT>
__device__ __forceinline__ void eliminate_slice(BlockSync &sy, const BlockLds<CONN> &G, uint8_t *s_st,
                                                const int16_t *s_lst, const int32_t *s_sum, int nf, int p0, int p1) {
    constexpr int ND = 2 * Sten<CONN>::H;
    int pn[MAXPT];
    int32_t ub[MAXPT], sb[MAXPT];
    int32_t cb[MAXPT][ND];   // capacity towards in-slice neighbours, 0 otherwise
DOPE_UNROLL
    for (int j = 0; j < MAXPT; ++j) {
        const int i = sy.idx + j * sy.step;
        pn[j] = -1;
        ub[j] = 0;
        sb[j] = 0;
DOPE_UNROLL
        for (int d = 0; d < ND; ++d) cb[j][d] = 0;
        if (i < nf) {
            const int p = s_lst[i];
            const DirMask<CONN> m = G.msk[p];
            pn[j] = p;
            ub[j] = G.dd[p];
            sb[j] = s_sum[i];
DOPE_UNROLL
            for (int d = 0; d < ND; ++d) {
                const int q = G.nbr(p, d);
                cb[j][d] = (((m >> d) & 1u) && q >= p0 && q < p1) ? G.capd(p, d) : 0;
            }
        }
    }
    for (;;) {
        int ch = 0;
        for (;;) {
            int wch = 0;
DOPE_UNROLL
            for (int j = 0; j < MAXPT; ++j) {
                const int p = pn[j];
                if (p < 0) continue;
                uint8_t sv[ND];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) sv[d] = s_st[(cb[j][d] ? G.nbr(p, d) : p) - p0];   // p for the rest
                int32_t U = ub[j], S = sb[j];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) {
                    const int32_t c = cb[j][d];
                    if (sv[d] & ST_FIXED) {
                        U += (sv[d] & ST_LABEL) ? -c : c;
                        S -= c;
                    }
                }
                if (U < -S) { s_st[p - p0] = ST_FIXED | ST_LABEL; pn[j] = -1; wch |= 1; }
                else if (U > S) { s_st[p - p0] = ST_FIXED; pn[j] = -1; wch |= 1; }
                else wch |= 2;
            }
            if (!__any(wch & 1)) {
                ch |= wch;
                break;
            }
            ch |= wch & 1;
        }
        if (!(sy.bits(ch) & 1)) return;
    }
}

// list entries per thread loaded together by the batched elimination of the global-memory variant
constexpr int ELIM_BATCH = 4;
// The two-launch global-memory solve (k_block_prep_gmem): at most PREP_SLICE_MAX nodes per slice and
// PREP_SLICES_MAX slices per block (their free counts fill int32 slots 1..8 of the block region's header).
constexpr int PREP_SLICE_MAX = 4096;
constexpr int PREP_SLICES_MAX = 8;
// Blocks of at most this many nodes keep the one-launch solver: the second launch and the copy of the node arrays
// cost more than the spread prologue gains there (64 blocks of 70x70 pixels, one iteration: 14 vs 18 us).
constexpr int PREP_MIN_NP = 8192;

// Keeps the list entries that are still free (order not preserved); returns their count.  The height array,
// not yet in use, holds the survivors by list position in between.  Whole workgroup; ctr is a zeroed LDS slot.
template <int CONN>
__device__ __forceinline__ int compact_free(BlockLds<CONN> &L, int nfree, int *ctr, int tid, int nt) {
    for (int i = tid; i < nfree; i += nt) {
        const int p = L.lst[i];
        L.hh[i] = (L.st[p] & ST_FIXED) ? int16_t(-1) : int16_t(p);
    }
    __syncthreads();
    for (int i = tid; i < nfree; i += nt) {
        const int v = L.hh[i];
        if (v >= 0) L.lst[atomicAdd(ctr, 1)] = int16_t(v);
    }
    __syncthreads();
    return *ctr;
}

// The nodes a thread visits in the flow phases: its entries idx, idx + step, ... of the LDS list (fixed nodes
// included, skipped at every visit) ...
struct LdsNodes {
    static constexpr bool FREE_ONLY = false;
    const int16_t *lst;
    int idx, step, n;
    template <class F>
    __device__ __forceinline__ void each(F &&f) const {
        for (int i = idx; i < n; i += step) f(int(lst[i]));
    }
    // f on the nodes for which pred holds
    template <class P, class F>
    __device__ __forceinline__ void each_where(P &&pred, F &&f) const {
        for (int i = idx; i < n; i += step) {
            const int p = lst[i];
            if (pred(p)) f(p);
        }
    }
};

// ... or the same entries held in registers (at most MAXPT per thread), the fixed ones dropped once: a visit then
// costs no list load, and the loads of a thread's nodes are independent of each other.
template <int MAXPT>
struct RegNodes {
    static constexpr bool FREE_ONLY = true;
    int p[MAXPT];
    int16_t *lst;
    int idx, step;
    __device__ __forceinline__ RegNodes(int16_t *lst_, const uint8_t *st, int idx_, int step_, int n)
        : lst(lst_), idx(idx_), step(step_) {
DOPE_UNROLL
        for (int j = 0; j < MAXPT; ++j) {
            const int i = idx + j * step;
            const int v = i < n ? int(lst[i]) : -1;
            p[j] = (v >= 0 && !(st[v] & ST_FIXED)) ? v : -1;
        }
    }
    template <class F>
    __device__ __forceinline__ void each(F &&f) const {
DOPE_UNROLL
        for (int j = 0; j < MAXPT; ++j)
            if (p[j] >= 0) f(p[j]);
    }
    // f on the nodes for which pred holds, spread over the lanes of the wavefront: the wavefront's candidates are
    // packed (ballot and prefix count) into its own list entries, which nothing reads once the nodes are held in
    // registers, and lane l takes candidates l, l + 64, ...  A sparse frontier or active set then costs the
    // wavefront one pass over its candidates instead of one pass per register slot in which any lane has one.
    // The entries used are the wavefront's first n positions in (slot, lane) order, all below the list length.
    template <class P, class F>
    __device__ __forceinline__ void each_where(P &&pred, F &&f) const {
        if constexpr (MAXPT == 1) {
            // one slot: the wavefront passes over it once whichever lanes hold candidates
            if (p[0] >= 0 && pred(p[0])) f(p[0]);
            return;
        }
        const int lane = idx & 63, wbase = idx - lane;
        int n = 0;
DOPE_UNROLL
        for (int j = 0; j < MAXPT; ++j) {
            const bool c = p[j] >= 0 && pred(p[j]);
            const unsigned long long bal = __ballot(c);
            if (c) {
                const int i = n + int(__builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32),
                                                                __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u)));
                lst[wbase + (i & 63) + (i >> 6) * step] = int16_t(p[j]);
            }
            n += __popcll(bal);
        }
        // the entries written by other lanes of this wavefront are read below
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i = lane; i < n; i += 64) f(int(lst[wbase + (i & 63) + (i >> 6) * step]));
    }
};

// Everything after the elimination for the nfree nodes of lst (visited through nodes): flow network, push-relabel
// to a max preflow, and the canonical cut (ST_MARK = label 1).
template <int CONN, class Sync, class Nodes>
__device__ __forceinline__ void flow_network(Sync &sy, BlockLds<CONN> &L, const Nodes &nodes, int nfree,
                                             int32_t round_limit, int32_t relabel_period, FlowStats &fs) {
    constexpr int ND = 2 * Sten<CONN>::H;
    auto fixed = [&](int p) -> bool { return !Nodes::FREE_ONLY && (L.st[p] & ST_FIXED); };
    // (2) flow network of the remaining free nodes: source excess -U and sink capacity U in one signed value
    nodes.each([&](int p) {
        if (fixed(p)) return;
        const DirMask<CONN> m = L.msk[p];
        DirMask<CONN> live = 0;
        int32_t U = L.dd[p];
DOPE_UNROLL
        for (int d = 0; d < ND; ++d)
            if ((m >> d) & 1u) {
                const uint8_t sv = L.st[L.nbr(p, d)];
                if (sv & ST_FIXED) U += (sv & ST_LABEL) ? -L.capd(p, d) : L.capd(p, d);
                else live |= DirMask<CONN>(1) << d;
            }
        L.msk[p] = LdsMask<CONN>(live);
        L.dd[p] = -U;
    });
    sy.sync();
    // (3) push-relabel with periodic global relabelling: heights become exact residual distances to the sink,
    //     by a breadth-first search backwards from the nodes with sink capacity left, one level per barrier.
    //     Level l's nodes (height l) hand l + 1 to every unlabelled neighbour with a residual arc into them, so a
    //     level costs each thread a look at its nodes' heights plus the arcs of the nodes on the frontier only.
    for (;;) {
        nodes.each([&](int p) {
            if (!fixed(p)) L.hh[p] = L.dd[p] < 0 ? 1 : H_INF;
        });
        sy.sync();
        for (int lvl = 1;; ++lvl) {
            bool grew = false;
            nodes.each_where([&](int p) { return L.hh[p] == lvl && !fixed(p); }, [&](int p) {
                const DirMask<CONN> m = L.msk[p];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d)
                    if ((m >> d) & 1u) {
                        const int v = L.nbr(p, d);
                        if (L.hh[v] == H_INF && L.res_in(p, d) > 0) {
                            L.hh[v] = int16_t(lvl + 1);
                            grew = true;
                        }
                    }
            });
            if (!sy.any(grew)) break;
        }
        bool act = false;
        nodes.each([&](int p) {
            if (!fixed(p) && L.dd[p] > 0 && L.hh[p] < H_INF) act = true;
        });
        if (!sy.any(act)) break;
        ++fs.grel;
        if (fs.rounds >= round_limit) { fs.fail = true; break; }
        for (int r = 0; r < relabel_period; ++r) {
            // push: heights are frozen, so an edge is admissible in one direction only; a node's excess only
            // grows until it pushes, so a node active when the active set is taken is still active here
            auto active = [&](int p) { return !fixed(p) && L.dd[p] > 0 && L.hh[p] < H_INF; };
            nodes.each_where(active, [&](int p) {
                const int32_t e = L.dd[p];
                const int h = L.hh[p];
                if (e <= 0 || h >= H_INF) return;
                const DirMask<CONN> m = L.msk[p];
                int32_t rem = e;
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) {
                    if (!((m >> d) & 1u) || rem == 0) continue;
                    const int v = L.nbr(p, d);
                    if (L.hh[v] != h - 1) continue;
                    const int32_t rs = L.res(p, d);
                    if (rs <= 0) continue;
                    const int32_t delta = rem < rs ? rem : rs;
                    L.push(p, d, delta);
                    atomicAdd(&L.dd[v], delta);
                    rem -= delta;
                }
                if (rem != e) atomicSub(&L.dd[p], e - rem);
            });
            sy.sync();
            // relabel: active nodes without an admissible arc rise to 1 + the lowest residual neighbour
            nodes.each_where(active, [&](int p) {
                const int h = L.hh[p];
                if (L.dd[p] <= 0 || h >= H_INF) return;
                const DirMask<CONN> m = L.msk[p];
                int best = 1 << 30;
                bool adm = false;
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) {
                    if (!((m >> d) & 1u) || adm) continue;
                    if (L.res(p, d) <= 0) continue;
                    const int hv = L.hh[L.nbr(p, d)];
                    if (hv == h - 1) adm = true;
                    else if (hv + 1 < best) best = hv + 1;
                }
                if (!adm) L.hh[p] = int16_t(best > nfree ? H_INF : best);   // no path of that length exists
            });
            sy.sync();
            ++fs.rounds;
        }
    }
    // (4) canonical cut: nodes reachable in the residual graph from any node holding excess, by a breadth-first
    //     search forwards from those nodes; the heights, no longer needed, hold the search levels (-1: not
    //     reached yet)
    nodes.each([&](int p) {
        if (fixed(p)) return;
        const bool ex = L.dd[p] > 0;
        L.hh[p] = ex ? int16_t(0) : int16_t(-1);
        if (ex) L.st[p] |= ST_MARK;
    });
    sy.sync();
    for (int lvl = 0;; ++lvl) {
        bool grew = false;
        nodes.each_where([&](int p) { return L.hh[p] == lvl && !fixed(p); }, [&](int p) {
            const DirMask<CONN> m = L.msk[p];
DOPE_UNROLL
            for (int d = 0; d < ND; ++d)
                if ((m >> d) & 1u) {
                    const int v = L.nbr(p, d);
                    if (L.hh[v] < 0 && L.res(p, d) > 0) {
                        L.hh[v] = int16_t(lvl + 1);
                        L.st[v] |= ST_MARK;
                        grew = true;
                    }
                }
        });
        if (!sy.any(grew)) break;
    }
#ifdef DOPE_DEBUG
    // (5) debug builds only: the marked set is the canonical cut of a maximum preflow -- every node holding
    //     excess is marked, no residual arc leaves the marked set, and no marked node has sink capacity left
    //     (dd < 0: an augmenting path from an excess) -- else the block reports a solver error
    bool bad = false;
    nodes.each([&](int p) {
        if (fixed(p)) return;
        const bool mk = (L.st[p] & ST_MARK) != 0;
        if (L.dd[p] > 0 && !mk) bad = true;
        if (!mk) return;
        if (L.dd[p] < 0) bad = true;
        const DirMask<CONN> m = L.msk[p];
DOPE_UNROLL
        for (int d = 0; d < ND; ++d)
            if (((m >> d) & 1u) && L.res(p, d) > 0 && !(L.st[L.nbr(p, d)] & ST_MARK)) bad = true;
    });
    if (sy.any(bad)) fs.fail = true;
#endif
}

// flow_network over the thread's list entries: held in registers when there are at most MAXPT per thread and the
// stencil has at most eight directions, otherwise (and always for MAXPT = 0) read from the LDS list at every visit.
template <int CONN, int MAXPT, class Sync>
__device__ __forceinline__ void flow_phases(Sync &sy, BlockLds<CONN> &L, int nfree, int32_t round_limit,
                                            int32_t relabel_period, FlowStats &fs) {
    if constexpr (2 * Sten<CONN>::H <= 8 && MAXPT > 0) {
        if (nfree <= MAXPT * sy.step) {
            const RegNodes<MAXPT> nodes(L.lst, L.st, sy.idx, sy.step, nfree);
            return flow_network<CONN>(sy, L, nodes, nfree, round_limit, relabel_period, fs);
        }
    }
    const LdsNodes nodes{L.lst, sy.idx, sy.step, nfree};
    flow_network<CONN>(sy, L, nodes, nfree, round_limit, relabel_period, fs);
}

// Free nodes up to this count are handled by one wavefront (wave-level synchronisation only).
constexpr int WAVE_FLOW_MAX = 64;

// Per-axis rows of log2 q of the block being solved (block_lq_rows): one array per kernel, shared by the variants
// of the block solve that a kernel inlines (a function-scope array would be allocated once per variant).
__shared__ uint16_t s_lq_rows[3][LQ_TAB];

// The per-node arrays of the maxflow_lds_bytes layout, starting noff bytes into base: unary / excess (4 B),
// height (2), free list (2), then the direction masks aligned to their size, then the state bytes.
template <int CONN>
__device__ __forceinline__ void bind_nodes(BlockLds<CONN> &L, unsigned char *base, size_t noff) {
    L.dd = reinterpret_cast<int32_t *>(base + noff);
    L.hh = reinterpret_cast<int16_t *>(L.dd + L.npmax);
    L.lst = L.hh + L.npmax;
    constexpr size_t MB = sizeof(LdsMask<CONN>);
    const size_t mo = noff + size_t(L.npmax) * 8;
    L.msk = reinterpret_cast<LdsMask<CONN> *>(base + ((mo + MB - 1) & ~(MB - 1)));
    L.st = reinterpret_cast<uint8_t *>(L.msk + L.npmax);
}

// Block k of the partition (closed form, no table load on the critical path) and its multiplier input.
struct BlockAt {
    int kx, ky, kz, x0, y0, z0, ex, ey, ez, np;
    int64_t off, M;
    double inv_ex, inv_ey;
    const GLOBAL int32_t *Ain;
};

__device__ __forceinline__ BlockAt block_place(const Img &im, int k, int parity) {
    const Geom &g = im.g;
    BlockAt b;
    b.kx = k % g.ax[0].nb;
    b.ky = (k / g.ax[0].nb) % g.ax[1].nb;
    b.kz = k / (g.ax[0].nb * g.ax[1].nb);
    b.x0 = b.kx * g.ax[0].s;
    b.y0 = b.ky * g.ax[1].s;
    b.z0 = b.kz * g.ax[2].s;
    b.ex = axis_ext(g.ax[0], b.kx);
    b.ey = axis_ext(g.ax[1], b.ky);
    b.ez = axis_ext(g.ax[2], b.kz);
    b.off = block_offset(g, b.kx, b.ky, b.kz);
    b.np = b.ex * b.ey * b.ez;
    b.Ain = gp(parity ? im.A1 : im.A0);
    b.M = gp(im.ctl)->M;
    b.inv_ex = axis_inv_ext(g.ax[0], b.kx);
    b.inv_ey = axis_inv_ext(g.ax[1], b.ky);
    return b;
}

// Prologue of the block solve over the block's nodes pbeg <= p < pend: Eq. (8) unaries, in-block capacities,
// strictly forced nodes (state, mask and unary into L's arrays), and the others appended to flst through the
// counter fctr.  fsum (when not null) receives each listed node's total in-block capacity at its list position,
// sst (when not null) every node's state at index p - pbeg.  walk: the caller's coordinate walk, set to
// pbeg + threadIdx.x with stride NT.
template <int CONN, int NT>
__device__ __forceinline__ void block_prologue(const Img &im, const BlockAt &b, BlockLds<CONN> &L, bool lq_tab,
                                               uint16_t (*s_lq)[LQ_TAB], LocalWalk &walk, int pbeg, int pend,
                                               int16_t *flst, int *fctr, int32_t *fsum, uint8_t *sst) {
    constexpr int H = Sten<CONN>::H;
    const Geom &g = im.g;
    const int npmax = L.npmax;
    const int x0 = b.x0, y0 = b.y0, z0 = b.z0, ex = b.ex, ey = b.ey, ez = b.ez;
    const int64_t off = b.off, M = b.M;
    const GLOBAL int32_t *Ain = b.Ain;
    const GLOBAL int32_t *gu = gp(im.u), *gcw = gp(im.cw), *gY = gp(im.Y);
    for (int p = pbeg + int(threadIdx.x); p < pend; p += NT, walk.next()) {
        const int3 l = make_int3(walk.lx, walk.ly, walk.lz);
        DirMask<CONN> m;
        int64_t sumc;
        int64_t Ut;
        if constexpr (2 * H > 48) {
            // the widest stencils (9x9, radius-3 and radius-4 balls): eight directions at a time, capacities
            // written as they come (holding all directions' gathers spilled hundreds of registers there; up to
            // the 7x7 square the one-shot gathers are faster)
            const uint32_t ci = uint32_t(off + p);
            const int gx = x0 + l.x, gy = y0 + l.y, gz = z0 + l.z;
            if (lq_tab) {
                const TabCov<CONN> tc{s_lq[0][l.x], s_lq[1][l.y], s_lq[2][l.z]};
                Ut = unary_chunked<CONN, 8>(g, gu, gcw, gY, Ain, ci, gx, gy, gz, tc, M, l.x, l.y, l.z, ex, ey, ez,
                                            L.cap + p, npmax, m, sumc);
            } else {
                BoxCov<CONN> bc;
                bc.init(g, gx, gy, gz);
                Ut = unary_chunked<CONN, 8>(g, gu, gcw, gY, Ain, ci, gx, gy, gz, bc, M, l.x, l.y, l.z, ex, ey, ez,
                                            L.cap + p, npmax, m, sumc);
            }
DOPE_UNROLL
            for (int o = 0; o < H; ++o) L.flw[o * npmax + p] = 0;
        } else {
            PixLoads<CONN> ld;
            unary_loads<CONN>(g, gu, gcw, gY, Ain, uint32_t(off + p), x0 + l.x, y0 + l.y, z0 + l.z, ld);
            int32_t cp[H];
            if (lq_tab) {
                const TabCov<CONN> tc{s_lq[0][l.x], s_lq[1][l.y], s_lq[2][l.z]};
                Ut = unary_from_cov<CONN>(tc, ld, M, l.x, l.y, l.z, ex, ey, ez, cp, m, sumc);
            } else {
                Ut = unary_from<CONN>(g, ld, M, x0 + l.x, y0 + l.y, z0 + l.z, l.x, l.y, l.z, ex, ey, ez, cp, m,
                                      sumc);
            }
DOPE_UNROLL
            for (int o = 0; o < H; ++o) {
                L.cap[o * npmax + p] = cp[o];
                L.flw[o * npmax + p] = 0;
            }
        }
        uint8_t sbits = 0;
        if (Ut < -sumc) sbits = ST_FIXED | ST_LABEL;       // label 1 in every minimiser
        else if (Ut > sumc) sbits = ST_FIXED;              // label 0 in every minimiser
        L.st[p] = sbits;
        if (sst) sst[p - pbeg] = sbits;
        L.msk[p] = LdsMask<CONN>(m);
        L.dd[p] = sbits ? 0 : int32_t(Ut);                 // |Ut| <= sumc < 2^29 for free nodes
        if (!sbits) {
            const int at = atomicAdd(fctr, 1);
            flst[at] = int16_t(p);
            if (fsum) fsum[at] = int32_t(sumc);
        }
    }
}

// par: multiplier buffer parity (t & 1), or -1 to read it from the loop control.  spec: the caller has not
// checked the loop control; the gathers are issued first and the block stops before its first global store when
// the iteration is skipped.  REGLIST: the flow phases may hold the thread's list entries in registers (the
// global-memory variant, short of registers already, reads them from the list).  SPLIT: the per-edge arrays
// (capacities and flows) live at gedge + 64 in global memory and only the per-node arrays in smem; otherwise the
// whole state lives in smem (the maxflow_lds_bytes layout).  STAGED (with SPLIT): k_block_prep_gmem has run the
// prologue and a first elimination already and left the whole maxflow_lds_bytes layout at gedge; the block copies
// the node arrays into smem and lists the nodes still free instead of running the prologue.
template <int CONN, int NT, bool REGLIST = true, bool SPLIT = false, bool STAGED = false>
__device__ __forceinline__ void block_maxflow(const Img &im, int k, unsigned char *smem, int32_t npmax,
                                              int32_t round_limit, int32_t relabel_period, int par, bool spec,
                                              unsigned char *gedge = nullptr) {
    constexpr int H = Sten<CONN>::H;
    static_assert(SPLIT || !STAGED, "the staged solve keeps its node arrays in smem");
    const Geom &g = im.g;
    const GLOBAL Ctl *ctl = gp(im.ctl);
    const int parity = par >= 0 ? par : (ctl->t & 1);
    // block geometry from the closed-form partition (no table load on the critical path)
    const int kx = k % g.ax[0].nb, ky = (k / g.ax[0].nb) % g.ax[1].nb, kz = k / (g.ax[0].nb * g.ax[1].nb);
    const int x0 = kx * g.ax[0].s, y0 = ky * g.ax[1].s, z0 = kz * g.ax[2].s;
    const int ex = axis_ext(g.ax[0], kx), ey = axis_ext(g.ax[1], ky), ez = axis_ext(g.ax[2], kz);
    const int64_t off = block_offset(g, kx, ky, kz);
    const int np = ex * ey * ez;
    const GLOBAL int32_t *Ain = gp(parity ? im.A1 : im.A0);
    const int64_t M = ctl->M;
    const int tid = threadIdx.x;

    // scalar slots 0..14: 1 free-list length, 2..4 barrier flags, 6..7 a 64-bit residual sum, 8 compaction count
    int *s_ctr = reinterpret_cast<int *>(smem);
    BlockLds<CONN> L;
    L.npmax = npmax;
    L.cap = reinterpret_cast<int32_t *>((SPLIT ? gedge : smem) + 64);
    L.flw = L.cap + H * npmax;
    // the node arrays follow the edge arrays, or start the LDS when the edge arrays are in global memory
    bind_nodes<CONN>(L, smem, SPLIT ? 64 : 64 + size_t(npmax) * 8 * H);
DOPE_UNROLL
    for (int o = 0; o < H; ++o) {
        const int3 v = half_off<CONN>(o);
        L.loff[o] = v.x + ex * (v.y + ey * v.z);
    }
    // covers of the block's coordinates, once per block (blocks of at most LQ_TAB pixels per axis)
    uint16_t (*s_lq)[LQ_TAB] = s_lq_rows;
    const bool lq_tab = !STAGED && ex <= LQ_TAB && ey <= LQ_TAB && ez <= LQ_TAB;   // uniform
    if (lq_tab) block_lq_rows<CONN, NT>(g, x0, y0, z0, ex, ey, ez, s_lq);
    if (tid < 15) s_ctr[tid] = 0;
    __syncthreads();

    const double inv_ex = axis_inv_ext(g.ax[0], kx), inv_ey = axis_inv_ext(g.ax[1], ky);
    LocalWalk walk;
    int nfree_stat = 0;   // free nodes after the prologue's forcing test (the statistics' count)
    if constexpr (STAGED) {
        // ---- the prologue kernel's node arrays into smem; list of the nodes its elimination left free ----
        // (four nodes per thread loaded before any is stored, so that their global loads overlap)
        BlockLds<CONN> G = L;
        bind_nodes<CONN>(G, gedge, 64 + size_t(npmax) * 8 * H);
        constexpr int CP = 4;
        for (int p0 = tid; p0 < np; p0 += CP * NT) {
            uint8_t sb[CP];
            LdsMask<CONN> mb[CP];
            int32_t db[CP];
DOPE_UNROLL
            for (int j = 0; j < CP; ++j) {
                const int p = p0 + j * NT;
                if (p < np) {
                    sb[j] = G.st[p];
                    mb[j] = G.msk[p];
                    db[j] = G.dd[p];
                }
            }
DOPE_UNROLL
            for (int j = 0; j < CP; ++j) {
                const int p = p0 + j * NT;
                if (p < np) {
                    L.st[p] = sb[j];
                    L.msk[p] = mb[j];
                    L.dd[p] = db[j];
                    if (!(sb[j] & ST_FIXED)) L.lst[atomicAdd(&s_ctr[1], 1)] = int16_t(p);
                }
            }
        }
        const GLOBAL int32_t *hdr = gp(reinterpret_cast<const int32_t *>(gedge));
        for (int s = 0; s < PREP_SLICES_MAX; ++s) nfree_stat += hdr[1 + s];
    } else {
        // ---- prologue: Eq. (8) unaries, in-block capacities, strictly forced nodes, list of the others ----
        const BlockAt b{kx, ky, kz, x0, y0, z0, ex, ey, ez, np, off, M, inv_ex, inv_ey, Ain};
        walk.init(tid, NT, ex, ey, inv_ex, inv_ey);
        block_prologue<CONN, NT>(im, b, L, lq_tab, s_lq, walk, 0, np, L.lst, &s_ctr[1], nullptr, nullptr);
    }
    __syncthreads();
    if (spec && ctl_skip(im.ctl)) return;   // uniform: every thread reads the same loop control
    const int nfree = s_ctr[1];
    if constexpr (!STAGED) nfree_stat = nfree;

    FlowStats fs{0, 0, 0, false};
    if (nfree > 0 && nfree <= WAVE_FLOW_MAX) {
        if (tid < 64) {
            WaveSync sy{tid, 64};
            if (eliminate_fast<CONN, 1>(sy, L, nfree, fs)) flow_phases<CONN, 1>(sy, L, nfree, round_limit, relabel_period, fs);
        }
    } else if (nfree > 0) {
        BlockSync sy{tid, NT, s_ctr + 2, 0};
        if (eliminate_fast<CONN, elim_regs<NT>(), BlockSync, REGLIST ? 0 : ELIM_BATCH>(sy, L, nfree, fs)) {
            // the flow phases only visit the nodes the elimination left free; few enough go to one wavefront
            const int nleft = compact_free<CONN>(L, nfree, s_ctr + 8, tid, NT);
            if (nleft <= WAVE_FLOW_MAX) {
                if (tid < 64) {
                    WaveSync ws{tid, 64};
                    flow_phases<CONN, 1>(ws, L, nleft, round_limit, relabel_period, fs);
                }
            } else {
                flow_phases<CONN, REGLIST ? elim_regs<NT>() : 0>(sy, L, nleft, round_limit, relabel_period, fs);
            }
        }
    }
    __syncthreads();

    // ---- labels; consensus and multipliers of the pixels interior to this block (Eq. 10 reduces to
    //      Y = 2^16 yhat + A and Eq. 11 to A = 0 there, and no other block reads them) ----
    GLOBAL int32_t *Aout = gp(parity ? im.A0 : im.A1);
    GLOBAL uint8_t *yhat = gp(im.yhat);
    GLOBAL uint8_t *yslot = gp(im.yslot);
    const int nslot = Sten<CONN>::NDIM == 3 ? 8 : 4;
    GLOBAL int32_t *Yg = gp(im.Y);
    unsigned long long r2 = 0;
    bool ovf = false;
    walk.init(tid, NT, ex, ey, inv_ex, inv_ey);
    for (int p = tid; p < np; p += NT, walk.next()) {
        const uint8_t sb = L.st[p];
        const int yv = (sb & ST_FIXED) ? ((sb & ST_LABEL) ? 1 : 0) : ((sb & ST_MARK) ? 1 : 0);
        const uint32_t cpy = uint32_t(off + p);
        st_at(yhat, cpy, uint8_t(yv));
        const int lx = walk.lx, ly = walk.ly, lz = walk.lz;
        const uint32_t m = uint32_t(x0 + lx) + uint32_t(g.W) * (uint32_t(y0 + ly) + uint32_t(g.H) * uint32_t(z0 + lz));
        st_at(yslot, m * uint32_t(nslot) + uint32_t(label_slot(g, kx, ky, kz, lx, ly, lz)), uint8_t(yv));
        if (is_interior(g, kx, ky, kz, x0 + lx, y0 + ly, z0 + lz)) {
            const int64_t Yn = int64_t(yv) * Y_ONE + ld_at(Ain, cpy << 2);
            if (Yn >= STATE_LIMIT || Yn <= -STATE_LIMIT) ovf = true;
            const int64_t Yc = Yn > STATE_LIMIT ? STATE_LIMIT : (Yn < -STATE_LIMIT ? -STATE_LIMIT : Yn);
            st_at(Yg, m << 2, int32_t(Yc));
            st_at(Aout, cpy << 2, int32_t(0));
            const int32_t rr = yv * Y_ONE - int32_t(Yc);   // |rr| < 2^23
            r2 += (unsigned long long)(int64_t(rr) * int64_t(rr));
        }
    }
    // r2 < 2^52 per lane (at most 16 pixels per thread, each square below 2^46)
    r2 = wave_sum64(r2);
    unsigned long long *s_r2 = reinterpret_cast<unsigned long long *>(s_ctr + 6);
    if ((tid & 63) == 63 && r2) atomicAdd(s_r2, r2);
    if (ovf) atomicOr((int32_t *)gp(&im.ctl->ovf_pending), 1);
    __syncthreads();
    if (tid == 0) {
        gp(im.resid)[k] = int64_t(*s_r2);    // the consensus kernel adds the other pixels of the block
        GLOBAL int32_t *st = gp(im.stats) + 4 * k;
        st[0] = nfree_stat;
        st[1] = fs.rounds;
        st[2] = fs.grel;
        st[3] = fs.casc;
        if (fs.fail) atomicOr((int32_t *)gp(&im.ctl->solver_err), 1);
    }
}

// The image descriptors of a batch are read-only while a launch runs; reading them through the constant address
// space marks the loads invariant.
#define CONSTANT __attribute__((address_space(4)))
__device__ __forceinline__ const Img &const_img(const Img *p) {
    return *(const Img *)(const CONSTANT Img *)p;
}

// The block-solve kernels ask for at least two wavefronts per SIMD (at most 256 VGPRs): with the 7x7 stencil's
// 256-thread workgroups that lets two blocks share a CU, as their LDS allows.
//
// Batch block solve, one workgroup per (image, block) item: workgroup b takes item b.  Items stay in dispatch
// order (round-robin over the XCDs): hard blocks cluster in space, and contiguous item ranges per XCD would leave
// XCDs idle behind the one that got the cluster.
template <int CONN, int NT>
__global__ __launch_bounds__(NT, 2) void k_block_solve(const Img *__restrict__ imgs, const Item *__restrict__ items,
                                                    int32_t npmax, int32_t round_limit, int32_t relabel_period) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Item wi = items[blockIdx.x];
    const Img &im = const_img(imgs + wi.img);
    if (!ctl_skip(im.ctl)) block_maxflow<CONN, NT>(im, wi.idx, smem, npmax, round_limit, relabel_period, -1, false);
}

// Persistent batch block solve: a fixed number of workgroups take (image, block) items from the device work queue
// until it is empty, so blocks of uneven max-flow cost balance over the workgroups.  A kernel of its own: the
// loop around the inlined solver raises register pressure, which the one-item-per-workgroup kernel need not pay.
template <int CONN, int NT>
__global__ __launch_bounds__(NT, 2) void k_block_solve_queue(const Img *__restrict__ imgs,
                                                             const Item *__restrict__ items,
                                                          int32_t n_items, Queue *queue, int32_t npmax,
                                                          int32_t round_limit, int32_t relabel_period) {
    extern __shared__ __align__(16) unsigned char smem[];
    int *s_item = reinterpret_cast<int *>(smem) + 15;   // the block solver uses scalar slots 0..14
    for (;;) {
        if (threadIdx.x == 0) *s_item = int(atomicAdd(&queue->next, 1u));
        __syncthreads();
        const int it = *s_item;
        __syncthreads();
        if (it >= n_items) break;
        const Item wi = items[it];
        const Img &im = const_img(imgs + wi.img);
        if (!ctl_skip(im.ctl)) block_maxflow<CONN, NT>(im, wi.idx, smem, npmax, round_limit, relabel_period, -1, false);
        __syncthreads();   // the LDS of this item is reused by the next one
    }
}

// One-image block solve: the image descriptor and the multiplier parity come as kernel arguments, and no
// descriptor or loop-control load stands between the launch and the gathers (the loop control is read while they
// are in flight; a skipped iteration stops before its first global store).  Workgroup b solves block
// block_at(g, b): the blocks of full extent first, each XCD taking a contiguous range of them, so the halo lines
// that neighbouring blocks share are fetched into one L2 (measured on MI355X: 7x7 neighbourhood 55 -> 41 us per
// launch, 5x5 30 -> 28 us, 512x512 8-connected solve 2 % faster), then the clipped blocks.  The batch kernels
// keep dispatch order, where whole images of hard blocks would otherwise land on one XCD.
template <int CONN, int NT>
__global__ __launch_bounds__(NT, 2) void k_block_solve_one(const Img one, int32_t par, int32_t npmax,
                                                        int32_t round_limit, int32_t relabel_period) {
    extern __shared__ __align__(16) unsigned char smem[];
    block_maxflow<CONN, NT>(one, block_at(one.g, blockIdx.x), smem, npmax, round_limit, relabel_period, par, true);
}

// One-image block solve for blocks whose max-flow state exceeds the LDS (large blocks of the paper's even
// partitions, or blocks of the wide stencils larger than a few hundred pixels): the same solver with its state in
// a global-memory region of the workgroup's own, scratch + b * stride (stride >= maxflow_lds_bytes(npmax, h)),
// which stays mostly in the L2.  split != 0: only the per-edge arrays (capacities and flows, 8h bytes per node)
// go there and the per-node arrays (excess, height, list, mask, state: 9 + m bytes per node) and the barrier slots
// stay in dynamic LDS; otherwise everything is in the region.  Barriers order the global accesses as they do LDS
// ones (workgroup-scope fences; the waves of a workgroup share one CU).
template <int CONN, int NT>
__global__ __launch_bounds__(NT, 2) void k_block_solve_gmem(const Img one, int32_t par, int32_t npmax,
                                                         int32_t round_limit, int32_t relabel_period,
                                                         unsigned char *scratch, uint64_t stride, int32_t split) {
    extern __shared__ __align__(16) unsigned char smem[];
    // a skipped iteration returns before the prologue, whose state would go to global memory
    if (ctl_skip(one.ctl)) return;
    unsigned char *mem = scratch + uint64_t(blockIdx.x) * stride;
    const int k = block_at(one.g, blockIdx.x);
    if (split)
        block_maxflow<CONN, NT, false, true>(one, k, smem, npmax, round_limit, relabel_period, par, false, mem);
    else
        block_maxflow<CONN, NT, false>(one, k, mem, npmax, round_limit, relabel_period, par, false);
}

// Blocks beyond the LDS with the 3x3 stencils, in two launches so that more than one CU works on each block's
// prologue (a partition of 128 large blocks would otherwise leave half the CUs idle while its prologue and
// elimination, most of the solve after the first iteration, run).  k_block_prep_gmem: workgroup w takes slice
// w / nb (of nslice) of block w % nb, runs the prologue over the slice's nodes into the whole maxflow_lds_bytes
// layout at the block's global region, then the elimination over the slice alone (eliminate_slice), and stores
// the slice's states and its prologue free count (int32 slot 1 + slice of the region's 64-byte header).
// k_block_flow_gmem then runs the rest of the block solve from that state, one workgroup per block.
template <int CONN, int NT>
__global__ __launch_bounds__(NT) void k_block_prep_gmem(const Img one, int32_t par, int32_t npmax,
                                                      unsigned char *scratch, uint64_t stride, int32_t nb,
                                                      int32_t nslice) {
    constexpr int H = Sten<CONN>::H;
    extern __shared__ __align__(16) unsigned char smem[];
    if (ctl_skip(one.ctl)) return;
    const int w = blockIdx.x, bi = w % nb, sl = w / nb;
    unsigned char *mem = scratch + uint64_t(bi) * stride;
    const int k = block_at(one.g, bi);
    const int parity = par >= 0 ? par : (gp(one.ctl)->t & 1);
    const BlockAt b = block_place(one, k, parity);
    const int p0 = int(int64_t(b.np) * sl / nslice), p1 = int(int64_t(b.np) * (sl + 1) / nslice);
    const int tid = threadIdx.x;
    // smem: 16 counters, the slice's list (int16) and capacity totals (int32), its states (bytes)
    int *s_ctr = reinterpret_cast<int *>(smem);
    int16_t *s_lst = reinterpret_cast<int16_t *>(smem + 64);
    int32_t *s_sum = reinterpret_cast<int32_t *>(smem + 64 + 2 * PREP_SLICE_MAX);
    uint8_t *s_st = smem + 64 + 6 * PREP_SLICE_MAX;
    BlockLds<CONN> G;
    G.npmax = npmax;
    G.cap = reinterpret_cast<int32_t *>(mem + 64);
    G.flw = G.cap + H * npmax;
    bind_nodes<CONN>(G, mem, 64 + size_t(npmax) * 8 * H);
DOPE_UNROLL
    for (int o = 0; o < H; ++o) {
        const int3 v = half_off<CONN>(o);
        G.loff[o] = v.x + b.ex * (v.y + b.ey * v.z);
    }
    uint16_t (*s_lq)[LQ_TAB] = s_lq_rows;
    const bool lq_tab = b.ex <= LQ_TAB && b.ey <= LQ_TAB && b.ez <= LQ_TAB;   // uniform
    if (lq_tab) block_lq_rows<CONN, NT>(one.g, b.x0, b.y0, b.z0, b.ex, b.ey, b.ez, s_lq);
    if (tid < 16) s_ctr[tid] = 0;
    __syncthreads();
    LocalWalk walk;
    walk.init(p0 + tid, NT, b.ex, b.ey, b.inv_ex, b.inv_ey);
    block_prologue<CONN, NT>(one, b, G, lq_tab, s_lq, walk, p0, p1, s_lst, &s_ctr[1], s_sum, s_st);
    __syncthreads();   // the slice's capacities (global) and states are complete for the workgroup
    const int nf = s_ctr[1];
    if (tid == 0) {
        GLOBAL int32_t *hdr = gp(reinterpret_cast<int32_t *>(mem));
        hdr[1 + sl] = nf;
        if (sl == 0)
            for (int s = nslice; s < PREP_SLICES_MAX; ++s) hdr[1 + s] = 0;
    }
    if (nf == 0) return;   // uniform; the prologue stored every state of the slice
    BlockSync sy{tid, NT, s_ctr + 2, 0};
    eliminate_slice<CONN, PREP_SLICE_MAX / NT>(sy, G, s_st, s_lst, s_sum, nf, p0, p1);
    __syncthreads();
    for (int i = tid; i < nf; i += NT) {
        const int p = s_lst[i];
        G.st[p] = s_st[p - p0];
    }
}

template <int CONN, int NT>
__global__ __launch_bounds__(NT) void k_block_flow_gmem(const Img one, int32_t par, int32_t npmax,
                                                      int32_t round_limit, int32_t relabel_period,
                                                      unsigned char *scratch, uint64_t stride) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (ctl_skip(one.ctl)) return;
    unsigned char *mem = scratch + uint64_t(blockIdx.x) * stride;
    const int k = block_at(one.g, blockIdx.x);
    block_maxflow<CONN, NT, false, true, true>(one, k, smem, npmax, round_limit, relabel_period, par, false, mem);
}

// ------------------------------------------------------------------------------------------------------------
// LSA-TR block solve: non-submodular blocks larger than enumeration allows (blocks that fit the LDS)
// ------------------------------------------------------------------------------------------------------------
//
// The trust-region local submodular approximation of Gorelick et al. (CVPR 2014), the non-submodular optimiser
// whose computations the paper distributes in its curvature experiment (Sec. 3.3).  The block problem is Eq. (8)
// scaled by 2^14 with capacities of either sign.  Each step linearises the supermodular terms (c < 0) at the
// current labelling x~ (c (1 - 2 x~_j) added to U_i for every edge (i, j) with c < 0), adds the trust region
// lam (1 - 2 x~_i) to U_i and solves the remaining submodular problem with the block max-flow (canonical minimal
// cut).  With R = E(x~) - E(x*) (actual) and P = A(x~) - A(x*) (predicted by the approximation), x* is accepted
// when R > 0 and 4 R >= P; a step that also has 4 R >= 3 P widens the region (lam level down), a rejected step
// narrows it (level up).  lam = 0 at level -1 and 2^14 10^k at level k; the search ends when x* = x~, when the level
// passes LSA_LEVEL_MAX or after LSA_MAX_STEPS steps.  Start: x~_i = [U_i < 0].

constexpr int64_t LSA_LAMBDA_UNIT = 1 << 14;
constexpr int LSA_LEVEL_MAX = 4;
constexpr int LSA_MAX_STEPS = 32;

__device__ __forceinline__ int64_t lsa_lambda(int level) {
    int64_t l = level >= 0 ? LSA_LAMBDA_UNIT : 0;
    for (int k = 0; k < level; ++k) l *= 10;
    return l;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
DOPE_UNROLL
    for (int s = 32; s >= 1; s >>= 1) x += __shfl_xor(x, s);
    return x;
}

// Label of node p in the solved step: forced nodes carry it in ST_LABEL, free nodes in ST_MARK (the minimal cut).
__device__ __forceinline__ int lsa_cand(uint8_t sb) {
    return (sb & ST_FIXED) ? ((sb & ST_LABEL) ? 1 : 0) : ((sb & ST_MARK) ? 1 : 0);
}

template <int CONN, int NT>
__device__ __forceinline__ void block_lsatr(const Img &im, int k, unsigned char *smem, int32_t npmax,
                                            int32_t round_limit, int32_t relabel_period) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    __shared__ long long s_rp[2];
    __shared__ int s_chg;
    const Geom &g = im.g;
    const GLOBAL Ctl *ctl = gp(im.ctl);
    const int parity = ctl->t & 1;
    const int kx = k % g.ax[0].nb, ky = (k / g.ax[0].nb) % g.ax[1].nb, kz = k / (g.ax[0].nb * g.ax[1].nb);
    const int x0 = kx * g.ax[0].s, y0 = ky * g.ax[1].s, z0 = kz * g.ax[2].s;
    const int ex = axis_ext(g.ax[0], kx), ey = axis_ext(g.ax[1], ky), ez = axis_ext(g.ax[2], kz);
    const int64_t off = block_offset(g, kx, ky, kz);
    const int np = ex * ey * ez;
    const GLOBAL int32_t *Ain = gp(parity ? im.A1 : im.A0);
    const int64_t M = ctl->M;
    const int tid = threadIdx.x;

    // max-flow state (as block_maxflow), then signed capacities, clamped unaries, all-edge masks and labels
    int *s_ctr = reinterpret_cast<int *>(smem);
    BlockLds<CONN> L;
    L.npmax = npmax;
    L.cap = reinterpret_cast<int32_t *>(smem + 64);
    L.flw = L.cap + H * npmax;
    L.dd = L.flw + H * npmax;
    L.hh = reinterpret_cast<int16_t *>(L.dd + npmax);
    L.lst = L.hh + npmax;
    constexpr size_t MB = sizeof(LdsMask<CONN>);
    {
        const size_t mo = 64 + size_t(npmax) * (8 * H + 8);
        L.msk = reinterpret_cast<LdsMask<CONN> *>(smem + ((mo + MB - 1) & ~(MB - 1)));
    }
    L.st = reinterpret_cast<uint8_t *>(L.msk + npmax);
    const size_t base = ((reinterpret_cast<size_t>(L.st + npmax) - reinterpret_cast<size_t>(smem)) + 15) & ~size_t(15);
    int32_t *csg = reinterpret_cast<int32_t *>(smem + base);              // [H][npmax] signed c (0 if absent)
    int32_t *u0 = csg + H * npmax;                                        // Eq. (8) unary clamped to int32
    LdsMask<CONN> *allm = reinterpret_cast<LdsMask<CONN> *>(u0 + npmax);  // in-block directions with c != 0
    uint8_t *xt = reinterpret_cast<uint8_t *>(allm + npmax);              // current labelling x~
DOPE_UNROLL
    for (int o = 0; o < H; ++o) {
        const int3 v = half_off<CONN>(o);
        L.loff[o] = v.x + ex * (v.y + ey * v.z);
    }

    // ---- prologue: Eq. (8) unaries and signed in-block capacities ----
    const GLOBAL int32_t *gu = gp(im.u), *gcw = gp(im.cw), *gY = gp(im.Y);
    const double inv_ex = axis_inv_ext(g.ax[0], kx), inv_ey = axis_inv_ext(g.ax[1], ky);
    for (int p = tid; p < np; p += NT) {
        const int3 l = block_local(p, ex, ey, inv_ex, inv_ey);
        PixLoads<CONN> ld;
        unary_loads<CONN>(g, gu, gcw, gY, Ain, uint32_t(off + p), x0 + l.x, y0 + l.y, z0 + l.z, ld);
        int32_t cp[H];
        DirMask<CONN> m;
        int64_t sumc;
        const int64_t Ut = unary_from<CONN>(g, ld, M, x0 + l.x, y0 + l.y, z0 + l.z, l.x, l.y, l.z, ex, ey, ez, cp, m,
                                            sumc);
DOPE_UNROLL
        for (int o = 0; o < H; ++o) csg[o * npmax + p] = cp[o];
        allm[p] = LdsMask<CONN>(m);
        u0[p] = int32_t(Ut > INT32_MAX ? int64_t(INT32_MAX) : (Ut < -int64_t(INT32_MAX) ? -int64_t(INT32_MAX) : Ut));
        xt[p] = Ut < 0 ? 1 : 0;
    }
    __syncthreads();

    FlowStats tot{0, 0, 0, false};
    int level = -1, steps = 0, nfree_last = 0;
    for (int step = 0; step < LSA_MAX_STEPS; ++step) {
        ++steps;
        const int64_t lam = lsa_lambda(level);
        if (tid < 15) s_ctr[tid] = 0;
        if (tid == 0) { s_rp[0] = 0; s_rp[1] = 0; s_chg = 0; }
        __syncthreads();
        // ---- step set-up: linearised and trust-region unaries, positive capacities, strict forcing ----
        for (int p = tid; p < np; p += NT) {
            const DirMask<CONN> am = allm[p];
            int64_t U1 = u0[p];
            int32_t splus = 0;
            DirMask<CONN> live = 0;
DOPE_UNROLL
            for (int d = 0; d < ND; ++d)
                if ((am >> d) & 1u) {
                    const int32_t c = d < H ? csg[d * npmax + p] : csg[(d - H) * npmax + p - L.loff[d - H]];
                    if (c < 0) {
                        U1 += int64_t(c) * (1 - 2 * int(xt[L.nbr(p, d)]));
                    } else {
                        splus += c;
                        live |= DirMask<CONN>(1) << d;
                    }
                }
            const int64_t U2 = U1 + lam * (1 - 2 * int(xt[p]));
DOPE_UNROLL
            for (int o = 0; o < H; ++o) {
                const int32_t c = csg[o * npmax + p];
                L.cap[o * npmax + p] = c > 0 ? c : 0;
                L.flw[o * npmax + p] = 0;
            }
            L.msk[p] = LdsMask<CONN>(live);
            uint8_t sb = 0;
            if (U2 < -int64_t(splus)) sb = ST_FIXED | ST_LABEL;
            else if (U2 > int64_t(splus)) sb = ST_FIXED;
            L.st[p] = sb;
            L.dd[p] = sb ? 0 : int32_t(U2);   // |U2| <= splus < 2^29 for free nodes
            if (!sb) L.lst[atomicAdd(&s_ctr[1], 1)] = int16_t(p);
        }
        __syncthreads();
        const int nfree = s_ctr[1];
        nfree_last = nfree;
        FlowStats fs{0, 0, 0, false};
        if (nfree > 0 && nfree <= WAVE_FLOW_MAX) {
            if (tid < 64) {
                WaveSync sy{tid, 64};
                if (eliminate_fast<CONN, 1>(sy, L, nfree, fs)) flow_phases<CONN, 1>(sy, L, nfree, round_limit, relabel_period, fs);
            }
        } else if (nfree > 0) {
            BlockSync sy{tid, NT, s_ctr + 2, 0};
            if (eliminate_fast<CONN, elim_regs<NT>()>(sy, L, nfree, fs)) {
                const int nleft = compact_free<CONN>(L, nfree, s_ctr + 8, tid, NT);
                if (nleft <= WAVE_FLOW_MAX) {
                    if (tid < 64) {
                        WaveSync ws{tid, 64};
                        flow_phases<CONN, 1>(ws, L, nleft, round_limit, relabel_period, fs);
                    }
                } else {
                    flow_phases<CONN, elim_regs<NT>()>(sy, L, nleft, round_limit, relabel_period, fs);
                }
            }
        }
        tot.rounds += fs.rounds;
        tot.grel += fs.grel;
        tot.casc += fs.casc;
        tot.fail = tot.fail || fs.fail;
        __syncthreads();
        // ---- actual and predicted reductions of the candidate ----
        int64_t eR = 0, eP = 0;
        int chg = 0;
        for (int p = tid; p < np; p += NT) {
            const int xo = xt[p], xn = lsa_cand(L.st[p]);
            const DirMask<CONN> am = allm[p];
            if (xo != xn) {
                chg = 1;
                int64_t U1 = u0[p];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d)
                    if ((am >> d) & 1u) {
                        const int32_t c = d < H ? csg[d * npmax + p] : csg[(d - H) * npmax + p - L.loff[d - H]];
                        if (c < 0) U1 += int64_t(c) * (1 - 2 * int(xt[L.nbr(p, d)]));
                    }
                eR += int64_t(u0[p]) * (xo - xn);
                eP += U1 * (xo - xn);
            }
DOPE_UNROLL
            for (int o = 0; o < H; ++o)
                if ((am >> o) & 1u) {
                    const int q = p + L.loff[o];
                    const int32_t c = csg[o * npmax + p];
                    const int qo = xt[q], qn = lsa_cand(L.st[q]);
                    const int t = (xo != qo ? 1 : 0) - (xn != qn ? 1 : 0);
                    if (t) {
                        eR += int64_t(c) * t;
                        if (c > 0) eP += int64_t(c) * t;
                    }
                }
        }
        eR = wave_sum_i64(eR);
        eP = wave_sum_i64(eP);
        chg = __any(chg) ? 1 : 0;
        if ((tid & 63) == 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&s_rp[0]), (unsigned long long)eR);
            atomicAdd(reinterpret_cast<unsigned long long *>(&s_rp[1]), (unsigned long long)eP);
            if (chg) atomicOr(&s_chg, 1);
        }
        __syncthreads();
        const int64_t R = s_rp[0], P = s_rp[1];
        if (!s_chg) break;                           // x* = x~: no better labelling in the region
        const bool accepted = R > 0 && 4 * R >= P;
        if (accepted) {
            for (int p = tid; p < np; p += NT) xt[p] = uint8_t(lsa_cand(L.st[p]));
            if (4 * R >= 3 * P && level >= 0) --level;
        } else {
            ++level;
        }
        __syncthreads();
        if (!accepted && level > LSA_LEVEL_MAX) break;
    }

    // ---- labels; consensus and multipliers of the pixels interior to this block (as block_maxflow) ----
    GLOBAL int32_t *Aout = gp(parity ? im.A0 : im.A1);
    GLOBAL uint8_t *yhat = gp(im.yhat);
    GLOBAL uint8_t *yslot = gp(im.yslot);
    const int nslot = Sten<CONN>::NDIM == 3 ? 8 : 4;
    GLOBAL int32_t *Yg = gp(im.Y);
    unsigned long long r2 = 0;
    bool ovf = false;
    for (int p = tid; p < np; p += NT) {
        const int yv = xt[p];
        const uint32_t cpy = uint32_t(off + p);
        st_at(yhat, cpy, uint8_t(yv));
        const int3 l = block_local(p, ex, ey, inv_ex, inv_ey);
        const int lx = l.x, ly = l.y, lz = l.z;
        const uint32_t m = uint32_t(x0 + lx) + uint32_t(g.W) * (uint32_t(y0 + ly) + uint32_t(g.H) * uint32_t(z0 + lz));
        st_at(yslot, m * uint32_t(nslot) + uint32_t(label_slot(g, kx, ky, kz, lx, ly, lz)), uint8_t(yv));
        if (is_interior(g, kx, ky, kz, x0 + lx, y0 + ly, z0 + lz)) {
            const int64_t Yn = int64_t(yv) * Y_ONE + ld_at(Ain, cpy << 2);
            if (Yn >= STATE_LIMIT || Yn <= -STATE_LIMIT) ovf = true;
            const int64_t Yc = Yn > STATE_LIMIT ? STATE_LIMIT : (Yn < -STATE_LIMIT ? -STATE_LIMIT : Yn);
            st_at(Yg, m << 2, int32_t(Yc));
            st_at(Aout, cpy << 2, int32_t(0));
            const int32_t rr = yv * Y_ONE - int32_t(Yc);   // |rr| < 2^23
            r2 += (unsigned long long)(int64_t(rr) * int64_t(rr));
        }
    }
    r2 = wave_sum64(r2);
    unsigned long long *s_r2 = reinterpret_cast<unsigned long long *>(s_ctr + 6);
    if (tid == 0) *s_r2 = 0;
    __syncthreads();
    if ((tid & 63) == 63 && r2) atomicAdd(s_r2, r2);
    if (ovf) atomicOr((int32_t *)gp(&im.ctl->ovf_pending), 1);
    __syncthreads();
    if (tid == 0) {
        gp(im.resid)[k] = int64_t(*s_r2);
        GLOBAL int32_t *st = gp(im.stats) + 4 * k;
        st[0] = nfree_last;
        st[1] = tot.rounds;
        st[2] = steps;
        st[3] = level;
        if (tot.fail) atomicOr((int32_t *)gp(&im.ctl->solver_err), 1);
    }
}

// LSA-TR block solve, one workgroup per (image, block) item (one image or a batch).
template <int CONN>
__global__ __launch_bounds__(LSATR_THREADS) void k_block_lsatr(const Img *__restrict__ imgs,
                                                               const Item *__restrict__ items, int32_t npmax,
                                                               int32_t round_limit, int32_t relabel_period) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Item wi = items[blockIdx.x];
    const Img &im = const_img(imgs + wi.img);
    if (!ctl_skip(im.ctl)) block_lsatr<CONN, LSATR_THREADS>(im, wi.idx, smem, npmax, round_limit, relabel_period);
}

// ------------------------------------------------------------------------------------------------------------
// Exhaustive block solve (blocks of at most 16 pixels, any sign of the weights)
// ------------------------------------------------------------------------------------------------------------

constexpr int EX_WAVES = 4;   // blocks per 256-thread workgroup

template <int CONN>
__global__ __launch_bounds__(256) void k_block_exhaustive(const Img *__restrict__ imgs,
                                                          const Item *__restrict__ items, int32_t n_items) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    __shared__ int32_t s_U[EX_WAVES][16];
    __shared__ int32_t s_nc[EX_WAVES][16][ND];   // capacity towards full-stencil neighbour d (0 = none)
    __shared__ int8_t s_nj[EX_WAVES][16][ND];    // local index of that neighbour
    __shared__ DirMask<CONN> s_m[EX_WAVES][16];  // in-block neighbour mask
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int it = blockIdx.x * EX_WAVES + wave;
    const Item wi = it < n_items ? items[it] : Item{0, 0};
    const Img &im = imgs[wi.img];
    const Geom &g = im.g;
    const Ctl *ctl = im.ctl;
    const int k = wi.idx;
    const bool live = it < n_items && !ctl_skip(ctl);
    int np = 0;
    int64_t off = 0;
    if (live) {
        const int32_t *bt = im.btab + BTAB_STRIDE * k;
        const int x0 = bt[0], y0 = bt[1], z0 = bt[2], ex = bt[3], ey = bt[4], ez = bt[5];
        off = bt[6];
        np = ex * ey * ez;
        const GLOBAL int32_t *Ain = gp((ctl->t & 1) ? im.A1 : im.A0);
        if (lane < np) {
            const int p = lane;
            const int lx = p % ex, r = p / ex, ly = r % ey, lz = r / ey;
            int32_t cp[H];
            DirMask<CONN> m;
            int64_t sumc;
            PixLoads<CONN> ld;
            unary_loads<CONN>(g, gp(im.u), gp(im.cw), gp(im.Y), Ain, uint32_t(off + p), x0 + lx, y0 + ly, z0 + lz,
                              ld);
            int64_t Ut = unary_from<CONN>(g, ld, gp(ctl)->M, x0 + lx, y0 + ly, z0 + lz, lx, ly, lz, ex, ey, ez, cp, m,
                                          sumc);
            // clamping a strictly forced unary to +-(sum |c| + 1) keeps the minimiser set
            if (Ut > sumc + 1) Ut = sumc + 1;
            if (Ut < -sumc - 1) Ut = -sumc - 1;
            s_U[wave][p] = int32_t(Ut);
            s_m[wave][p] = m;
DOPE_UNROLL
            for (int d = 0; d < ND; ++d) {
                const int3 v = full_dir<CONN>(d);
                // an absent neighbour points at the pixel itself with capacity 0, so the enumeration can use
                // every direction without a test
                const bool inb = (m >> d) & 1u;
                s_nj[wave][p][d] = int8_t(inb ? p + v.x + ex * (v.y + ey * v.z) : p);
                s_nc[wave][p][d] = (d < H && inb) ? cp[d] : 0;
            }
        }
    }
    __syncthreads();
    // the capacity towards a negative direction is the neighbour's positive half-edge
    if (live && lane < np) {
        const int p = lane;
        const DirMask<CONN> m = s_m[wave][p];
DOPE_UNROLL
        for (int d = H; d < ND; ++d)
            if ((m >> d) & 1u) s_nc[wave][p][d] = s_nc[wave][s_nj[wave][p][d]][d - H];
    }
    __syncthreads();
    if (!live) return;
    const int L = np > 6 ? np - 6 : 0;               // enumerated low bits per lane
    const int lanes_used = 1 << (np - L);
    // The minimiser with the smallest code is the smallest key E * 2^16 + code (codes are below 2^16 and
    // |E| < 2^35), so one 64-bit minimum keeps both the energy order and the tie rule.
    int64_t best = INT64_MAX;
    if (lane < lanes_used) {
        uint32_t x = uint32_t(lane) << L;
        int64_t E = 0;
        for (int p = 0; p < np; ++p) {
            const int xp = (x >> p) & 1;
            if (xp) E += s_U[wave][p];
DOPE_UNROLL
            for (int d = 0; d < H; ++d) {
                const int32_t c = s_nc[wave][p][d];
                if (c != 0) {
                    const int q = s_nj[wave][p][d];
                    if (xp != int((x >> q) & 1)) E += c;
                }
            }
        }
        int64_t key = E * 65536 + int64_t(x);
        best = key;
        const uint32_t cnt = 1u << L;
        // Gray-code step gi flips bit b = ctz(gi); E changes by +-t with t = U_b + sum_j (x_j ? -c_bj : c_bj)
        // = S_b - 2 sum_j (x_j ? c_bj : 0), S_b = U_b + sum_j c_bj, all below 2^31 in magnitude (|U_b| <= sum |c|
        // + 1 after the clamp above, sum |c| < 2^29); the key changes by +-(t 2^16 + 2^b)
        auto flip = [&](int b, int32_t sb, const int32_t *cb, const int *jb) {
            int32_t acc = 0;
DOPE_UNROLL
            for (int d = 0; d < ND; ++d) acc += cb[d] & -int32_t((x >> jb[d]) & 1u);
            const int64_t dk = int64_t(sb - 2 * acc) * 65536 + (int64_t(1) << b);
            key += ((x >> b) & 1u) ? -dk : dk;
            x ^= 1u << b;
            best = key < best ? key : best;
        };
        auto flip_lds = [&](int b) {
            int32_t cb[ND];
            int jb[ND];
            int32_t sb = s_U[wave][b];
DOPE_UNROLL
            for (int d = 0; d < ND; ++d) {
                cb[d] = s_nc[wave][b][d];
                jb[d] = s_nj[wave][b][d];
                sb += cb[d];
            }
            flip(b, sb, cb, jb);
        };
        constexpr int RB = 4;   // low bits whose data stays in registers
        if (ND <= 8 && L >= RB) {
            // fifteen of every sixteen steps flip one of bits 0..3 (ruler sequence 0 1 0 2 0 1 0 3 0 1 0 2 0 1 0,
            // then ctz >= 4): their data stays in registers, so one step in sixteen reads the block's LDS tables
            int32_t sr[RB], cr[RB][ND];
            int jr[RB][ND];
DOPE_UNROLL
            for (int b = 0; b < RB; ++b) {
                sr[b] = s_U[wave][b];
DOPE_UNROLL
                for (int d = 0; d < ND; ++d) {
                    cr[b][d] = s_nc[wave][b][d];
                    jr[b][d] = s_nj[wave][b][d];
                    sr[b] += cr[b][d];
                }
            }
            for (uint32_t gb = 0; gb < cnt; gb += 16) {
DOPE_UNROLL
                for (int i = 1; i < 16; ++i) {
                    const int b = __builtin_ctz(i);
                    flip(b, sr[b], cr[b], jr[b]);
                }
                if (gb + 16 < cnt) flip_lds(__builtin_ctz(gb + 16));
            }
        } else {
            for (uint32_t gi = 1; gi < cnt; ++gi) flip_lds(__builtin_ctz(gi));
        }
    }
DOPE_UNROLL
    for (int s = 32; s >= 1; s >>= 1) {
        const int64_t o = __shfl_xor(best, s);
        best = o < best ? o : best;
    }
    const uint32_t bestc = uint32_t(best & 0xFFFF);
    unsigned long long r2 = 0;
    if (lane < np) {
        const int yv = int((bestc >> lane) & 1u);
        gp(im.yhat)[off + lane] = uint8_t(yv);
        const int32_t *bt = im.btab + BTAB_STRIDE * k;
        const int ex = bt[3], ey = bt[4];
        const int lx = lane % ex, r = lane / ex, ly = r % ey, lz = r / ey;
        const int tx = k % g.ax[0].nb, ty = (k / g.ax[0].nb) % g.ax[1].nb, tz = k / (g.ax[0].nb * g.ax[1].nb);
        const int nslot = Sten<CONN>::NDIM == 3 ? 8 : 4;
        gp(im.yslot)[lin(g, bt[0] + lx, bt[1] + ly, bt[2] + lz) * nslot + label_slot(g, tx, ty, tz, lx, ly, lz)] =
            uint8_t(yv);
        if (is_interior(g, tx, ty, tz, bt[0] + lx, bt[1] + ly, bt[2] + lz)) {
            const GLOBAL int32_t *Ain = gp((ctl->t & 1) ? im.A1 : im.A0);
            GLOBAL int32_t *Aout = gp((ctl->t & 1) ? im.A0 : im.A1);
            const int64_t Yn = int64_t(yv) * Y_ONE + Ain[off + lane];
            if (Yn >= STATE_LIMIT || Yn <= -STATE_LIMIT) atomicOr((int32_t *)gp(&im.ctl->ovf_pending), 1);
            const int64_t Yc = Yn > STATE_LIMIT ? STATE_LIMIT : (Yn < -STATE_LIMIT ? -STATE_LIMIT : Yn);
            gp(im.Y)[lin(g, bt[0] + lx, bt[1] + ly, bt[2] + lz)] = int32_t(Yc);
            Aout[off + lane] = 0;
            const int64_t rr = int64_t(yv) * Y_ONE - Yc;
            r2 = (unsigned long long)(rr * rr);
        }
    }
DOPE_UNROLL
    for (int sft = 32; sft >= 1; sft >>= 1) r2 += __shfl_xor(r2, sft);
    if (lane == 0) {
        gp(im.resid)[k] = int64_t(r2);
        GLOBAL int32_t *st = gp(im.stats) + 4 * k;
        st[0] = np;
        st[1] = 0;
        st[2] = 0;
        st[3] = 0;
    }
}

// ------------------------------------------------------------------------------------------------------------
// Consensus (Eq. 10), multipliers (Eq. 11), residual and loop control
// ------------------------------------------------------------------------------------------------------------

constexpr int CONS_NT = CHUNK;   // boundary pixels per workgroup
constexpr int CONS_SPAN = 64;    // owner blocks of a chunk with residual slots in LDS

// One thread per boundary pixel m (a pixel that is not interior to its block), listed through its owner copy:
// the copy in the block with the highest index along every axis.  The thread gathers yhat and A of every copy
// of m and yhat of every copy of its stencil neighbours, computes Y_m (Eq. 10) once, writes it, writes the
// multiplier of every copy of m (Eq. 11), and adds (2^16 yhat_k,m - Y_m)^2 to r_k of each copy's block through
// LDS slots (owner block, copy) that are flushed with one global atomic per slot.
template <int CONN>
__device__ __forceinline__ void consensus_chunk(const Img &im, int chunk, int par, bool spec) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    constexpr int NDIM = Sten<CONN>::NDIM;
    constexpr int MAXC = 1 << NDIM;   // most blocks a pixel can lie in
    const Geom &g = im.g;
    const int tid = threadIdx.x;
    // the boundary-list record first: every gather of the pixel waits on it, the loop control does not
    const int64_t li = int64_t(chunk) * CONS_NT + tid;
    const bool in_list = li < im.n_blist;
    const uint64_t rec = in_list ? gp(reinterpret_cast<const uint64_t *>(im.blist))[li] : 0;
    const GLOBAL Ctl *ctl = gp(im.ctl);
    if (!spec && ctl_skip(im.ctl)) return;
    // speculative chunk: the loop control is read here but only the stores wait for it
    const bool skip = spec && ctl_skip(im.ctl);
    GLOBAL int32_t *__restrict__ Y = gp(im.Y);
    // slot (owner block - kfirst) * MAXC + copy for the first CONS_SPAN owner blocks of the chunk (a chunk of
    // boundary pixels listed by owner block rarely spans more; later owners add to the global residuals directly)
    __shared__ unsigned long long s_res[CONS_SPAN * MAXC];
    __shared__ unsigned long long s_tr[CONS_NT / 64][MAXC][64];   // per wavefront: residual of copy q by lane
    __shared__ int s_ovf;
    if (par < 0) par = ctl->t & 1;
    const GLOBAL int32_t *Ain = gp(par ? im.A1 : im.A0);
    GLOBAL int32_t *Aout = gp(par ? im.A0 : im.A1);
    const int64_t M = ctl->M;
    const double invM = 1.0 / double(M);
    const Axis &AX = g.ax[0], &AY = g.ax[1], &AZ = g.ax[2];
    const int kfirst = gp(im.chunk_k0)[chunk];
DOPE_UNROLL
    for (int q = 0; q < CONS_SPAN * MAXC / CONS_NT; ++q) s_res[q * CONS_NT + tid] = 0;
    if (tid == 0) s_ovf = 0;
    __syncthreads();
    int ovf = 0;
    int kk = kfirst;
    unsigned long long r2[MAXC];
DOPE_UNROLL
    for (int q = 0; q < MAXC; ++q) r2[q] = 0;
    if (in_list) {
        // the owner copy and its block (the record's two int32, copy first); the coordinates follow from the
        // closed-form block layout
        const int32_t c = int32_t(uint32_t(rec));
        kk = int32_t(uint32_t(rec >> 32));
        int kx, ky;
        const int kyz = qdiv(kk, AX.nb, AX.inv_nb, kx);
        const int kz = qdiv(kyz, AY.nb, AY.inv_nb, ky);
        const int ex = axis_ext(AX, kx), ey = axis_ext(AY, ky);
        const int p = int(c - block_offset(g, kx, ky, kz));
        const int3 l = block_local(p, ex, ey, axis_inv_ext(AX, kx), axis_inv_ext(AY, ky));
        const int gx = kx * AX.s + l.x, gy = ky * AY.s + l.y, gz = kz * AZ.s + l.z;
        const int32_t m = int32_t(lin(g, gx, gy, gz));
        // block intervals of the coordinates x - R .. x + R along each axis
        BoxCov<CONN> bc;
        if constexpr (Sten<CONN>::R == 1) bc.init_rows(gp(reinterpret_cast<const uint64_t *>(im.axrow)), g, gx, gy, gz);
        else bc.init(g, gx, gy, gz);
        const AxCov mx = bc.cx(0), my = bc.cy(0), mz = bc.cz(0);   // m itself
        const int lqm = bc.lq(make_int3(0, 0, 0));   // q_m = 2^lqm
        // Block-major index of pixel (x, y, z) in block (tx, ty, tz).  Indices are below 2^30 (sum of block
        // sizes), so the index is computed for every candidate block in wrapping 32-bit arithmetic and replaced
        // by the owner copy's index when that block does not exist: every gather is issued unconditionally and
        // masked afterwards, with no branch between the gathers.
        const uint32_t s0 = uint32_t(g.span[0]), s1 = uint32_t(g.span[1]);
        auto copy_at = [&](bool valid, int tx, int ty, int tz, int x, int y, int z) -> uint32_t {
            const uint32_t ex_t = uint32_t(axis_ext(AX, tx)), ey_t = uint32_t(axis_ext(AY, ty));
            const uint32_t ez_t = uint32_t(axis_ext(AZ, tz));
            const uint32_t boff = uint32_t(tz) * uint32_t(AZ.B) * s1 * s0 +
                                  ez_t * (uint32_t(ty) * uint32_t(AY.B) * s0 + ey_t * uint32_t(tx) * uint32_t(AX.B));
            const uint32_t cc = boff + uint32_t(x - tx * AX.s) +
                                ex_t * (uint32_t(y - ty * AY.s) + ey_t * uint32_t(z - tz * AZ.s));
            uint32_t r = valid ? cc : uint32_t(c);
            // optimisation barrier only (no instruction): keeps the compiler from turning the select back into a
            // branch around the load, which would serialise the gathers
            asm("" : "+v"(r));
            return r;
        };
        // ---- every load of this pixel is issued before any of them is used: the multipliers of its copies
        //      (block-major), its label slots and those of its stencil neighbours, and c_mj ----
        using SlotWord = typename std::conditional<MAXC == 8, uint64_t, uint32_t>::type;
        const GLOBAL SlotWord *ysl = reinterpret_cast<const GLOBAL SlotWord *>(gp(im.yslot));
        int32_t a_own[MAXC];
        uint32_t cc_own[MAXC];
        bool v_own[MAXC];
DOPE_UNROLL
        for (int q = 0; q < MAXC; ++q) {
            const int e = q & 1, b = (q >> 1) & 1, a = q >> 2;
            v_own[q] = e < mx.cnt && b < my.cnt && a < mz.cnt;
            cc_own[q] = copy_at(v_own[q], mx.thi - e, my.thi - b, mz.thi - a, gx, gy, gz);
            a_own[q] = ld_at(Ain, cc_own[q] << 2);
        }
        constexpr int WSH = MAXC == 8 ? 3 : 2;   // log2 of the label word size
        SlotWord wm = ld_at(ysl, uint32_t(m) << WSH);
        const DirMask<CONN> ingm = inside_mask<CONN>(gx, gy, gz, g.W, g.H, g.D);
        // c_mj and the label word of stencil neighbour d (an off-grid neighbour reads pixel m itself; its c is
        // masked where it is used)
        auto gather = [&](int d, int32_t &cv, SlotWord &w) {
            const int3 v = full_dir<CONN>(d);
            const int32_t dl = v.x + g.W * (v.y + g.H * v.z);
            uint32_t j = ((ingm >> d) & 1u) ? uint32_t(m) + uint32_t(dl) : uint32_t(m);
            asm("" : "+v"(j));   // optimisation barrier only: keeps the loads unconditional
            const GLOBAL int32_t *cwd = gp(im.cw) + int64_t(d < H ? d : d - H) * g.n;
            cv = ld_at(cwd, (d < H ? uint32_t(m) : j) << 2);
            w = ld_at(ysl, j << WSH);
        };
        // The label words hold one byte (0 or 1) per slot q = e + 2b + 4a.  A slot set along one axis is a byte
        // mask: slot bit e of that axis allowed for e in the 2-bit set.  A neighbour's copy in the block that is
        // m's slot q sits in the neighbour's slot q + (dx + 2dy + 4dz), d_ the difference of the two pixels'
        // top blocks, so shifting its word by that many bytes aligns the blocks holding both pixels.
        auto sel = [](int set, SlotWord lo, SlotWord hi) -> SlotWord {
            return ((set & 1) ? lo : SlotWord(0)) | ((set & 2) ? hi : SlotWord(0));
        };
        // every byte of a label word is 0 or 1, so the sum of its bytes is its population count
        auto bytesum = [](SlotWord x) -> int { return MAXC == 8 ? __popcll(uint64_t(x)) : __popc(uint32_t(x)); };
        const SlotWord X0 = MAXC == 8 ? SlotWord(0x00FF00FF00FF00FFull) : SlotWord(0x00FF00FFu);
        const SlotWord Y0 = MAXC == 8 ? SlotWord(0x0000FFFF0000FFFFull) : SlotWord(0x0000FFFFu);
        const SlotWord Z0 = MAXC == 8 ? SlotWord(0x00000000FFFFFFFFull) : SlotWord(0xFFFFFFFFu);
        const SlotWord X1 = SlotWord(~X0), Y1m = SlotWord(~Y0), Z1 = MAXC == 8 ? SlotWord(~Z0) : SlotWord(0);
        // slots e of one axis with e < cnt
        auto cnt_set = [](int cnt) -> int { return cnt >= 2 ? 3 : cnt; };
        // slots e of m's axis interval whose block also holds the neighbour (top differs by dt, neighbour count cn)
        auto shared_set = [](int cm, int dt, int cn) -> int {
            int set = 0;
DOPE_UNROLL
            for (int e = 0; e < 2; ++e)
                if (e < cm && e + dt >= 0 && e + dt < cn) set |= 1 << e;
            return set;
        };
        // the bracket of Hc for neighbour j (covers ax, ay, az along the axes, label word wjd, q_j = 2^lqj):
        // Y1 q_j - q_m (labels of j) - (labels of m minus labels of j over the blocks holding both), |.| <= 128
        auto hc_bracket = [&](const AxCov &ax, const AxCov &ay, const AxCov &az, SlotWord wjd, int lqj,
                              int Y1) -> int {
            const SlotWord vj = sel(cnt_set(ax.cnt), X0, X1) & sel(cnt_set(ay.cnt), Y0, Y1m) &
                                sel(cnt_set(az.cnt), Z0, Z1);
            const int yj_sum = bytesum(wjd & vj);
            const int dx = ax.thi - mx.thi, dy = ay.thi - my.thi, dz = az.thi - mz.thi;
            const SlotWord sm = sel(shared_set(mx.cnt, dx, ax.cnt), X0, X1) &
                                sel(shared_set(my.cnt, dy, ay.cnt), Y0, Y1m) &
                                sel(shared_set(mz.cnt, dz, az.cnt), Z0, Z1);
            const int sh = dx + 2 * dy + 4 * dz;
            // shift right by sh bytes when sh >= 0, left by -sh bytes otherwise (two shifts, no branch)
            const SlotWord wal = SlotWord(SlotWord(wjd >> (8 * (sh > 0 ? sh : 0))) << (8 * (sh < 0 ? -sh : 0)));
            const int shared = bytesum(wm & sm) - bytesum(wal & sm);
            // q_j and q_m are powers of two (an off-grid neighbour has c = 0, so its shift count does not matter)
            return (Y1 << lqj) - (yj_sum << lqm) - shared;
        };
        // ---- S_m and Hc_m.  With Y1 = sum of this pixel's labels, Hc regroups exactly as
        //      Hc = Y1 sum_j c_mj q_j - q_m sum_j c_mj (sum of j's labels)
        //           - sum_j c_mj sum_{blocks b holding m and j} (yhat_b,m - yhat_b,j) ----
        int32_t S = 0;   // at most 8 copies of 2^16 + 2^22 in magnitude: fits 32 bits
        int Y1 = 0;
        int yv_own[MAXC];
        int64_t HC = 0;
        if constexpr (ND <= 80) {
            // every gather of this pixel is issued before any of them is used
            int32_t cwv[ND];
            SlotWord wj[ND];
DOPE_UNROLL
            for (int d = 0; d < ND; ++d) gather(d, cwv[d], wj[d]);
            // optimisation barrier only: every gathered value is used after all gathers are issued
            if constexpr (CONN == 4) {
                asm("" : "+v"(a_own[0]), "+v"(a_own[1]), "+v"(a_own[2]), "+v"(a_own[3]), "+v"(wm), "+v"(cwv[0]),
                    "+v"(cwv[1]), "+v"(cwv[2]), "+v"(cwv[3]), "+v"(wj[0]), "+v"(wj[1]), "+v"(wj[2]), "+v"(wj[3]));
            } else if constexpr (CONN == 8) {
                asm("" : "+v"(a_own[0]), "+v"(a_own[1]), "+v"(a_own[2]), "+v"(a_own[3]), "+v"(wm), "+v"(cwv[0]),
                    "+v"(cwv[1]), "+v"(cwv[2]), "+v"(cwv[3]), "+v"(cwv[4]), "+v"(cwv[5]), "+v"(cwv[6]),
                    "+v"(cwv[7]), "+v"(wj[0]), "+v"(wj[1]), "+v"(wj[2]), "+v"(wj[3]), "+v"(wj[4]), "+v"(wj[5]),
                    "+v"(wj[6]), "+v"(wj[7]));
            } else if constexpr (CONN == 6) {
                asm("" : "+v"(a_own[0]), "+v"(a_own[1]), "+v"(a_own[2]), "+v"(a_own[3]), "+v"(a_own[4]),
                    "+v"(a_own[5]), "+v"(a_own[6]), "+v"(a_own[7]), "+v"(wm), "+v"(cwv[0]), "+v"(cwv[1]),
                    "+v"(cwv[2]), "+v"(cwv[3]), "+v"(cwv[4]), "+v"(cwv[5]), "+v"(wj[0]), "+v"(wj[1]), "+v"(wj[2]),
                    "+v"(wj[3]), "+v"(wj[4]), "+v"(wj[5]));
            }
DOPE_UNROLL
            for (int q = 0; q < MAXC; ++q) {
                yv_own[q] = v_own[q] ? int((wm >> (8 * q)) & 1u) : 0;
                if (!v_own[q]) a_own[q] = 0;
                S += yv_own[q] * Y_ONE + a_own[q];
                Y1 += yv_own[q];
            }
DOPE_UNROLL
            for (int d = 0; d < ND; ++d) {
                const int3 v = full_dir<CONN>(d);
                const int32_t c = ((ingm >> d) & 1u) ? cwv[d] : 0;
                HC += int64_t(c) * hc_bracket(bc.cx(v.x), bc.cy(v.y), bc.cz(v.z), wj[d], bc.lq(v), Y1);
            }
        } else {
            // the radius-3 and radius-4 balls: eight neighbours at a time (all of them at once held two values
            // per direction in private memory), their covers read from packed per-axis codes, so that no array is
            // indexed by a direction that is not a compile-time constant (up to the 9x9 square, 80 directions,
            // the one-shot gathers are faster)
DOPE_UNROLL
            for (int q = 0; q < MAXC; ++q) {
                yv_own[q] = v_own[q] ? int((wm >> (8 * q)) & 1u) : 0;
                if (!v_own[q]) a_own[q] = 0;
                S += yv_own[q] * Y_ONE + a_own[q];
                Y1 += yv_own[q];
            }
            constexpr int R = Sten<CONN>::R;
            // per axis, 4 bits per offset t = -R..R: cover count (2 bits) and top block minus m's top plus 1
            auto pack = [&](const AxCov *c, int top) -> uint64_t {
                uint64_t w = 0;
#pragma unroll
                for (int t = 0; t <= 2 * R; ++t)
                    w |= uint64_t((c[t].cnt & 3) | (((c[t].thi - top + 1) & 3) << 2)) << (4 * t);
                return w;
            };
            const uint64_t px = pack(bc.x, mx.thi), py = pack(bc.y, my.thi), pz = pack(bc.z, mz.thi);
            auto cov = [](uint64_t w, int off, int top) -> AxCov {
                const int code = int((w >> (4 * (off + R))) & 15u);
                return AxCov{top + ((code >> 2) & 3) - 1, code & 3};
            };
#pragma nounroll
            for (int d0 = 0; d0 < ND; d0 += 8) {
                int32_t cv[8];
                SlotWord w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) gather(d0 + j < ND ? d0 + j : ND - 1, cv[j], w[j]);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int d = d0 + j;
                    if (d >= ND) break;
                    const int3 v = full_dir<CONN>(d);
                    const AxCov ax = cov(px, v.x, mx.thi), ay = cov(py, v.y, my.thi), az = cov(pz, v.z, mz.thi);
                    const int lqj = max(ax.cnt - 1, 0) + max(ay.cnt - 1, 0) + max(az.cnt - 1, 0);
                    const int32_t c = ((ingm >> d) & 1u) ? cv[j] : 0;
                    HC += int64_t(c) * hc_bracket(ax, ay, az, w[j], lqj, Y1);
                }
            }
        }
        // floor((M S - 4 Hc) / (M q)) = floor(floor((M S - 4 Hc) / M) / q), q a power of two
        int64_t Yn = floor_div_est(M * int64_t(S) - 4 * HC, M, invM);
        Yn >>= lqm;
        if (Yn >= STATE_LIMIT || Yn <= -STATE_LIMIT) ovf = 1;
        const int64_t Yc = Yn > STATE_LIMIT ? STATE_LIMIT : (Yn < -STATE_LIMIT ? -STATE_LIMIT : Yn);
        if (!skip) st_at(Y, uint32_t(m) << 2, int32_t(Yc));
        // multipliers (Eq. 11) and residual terms of every copy
DOPE_UNROLL
        for (int q = 0; q < MAXC; ++q) {
            if (!v_own[q]) continue;
            const int64_t An = int64_t(a_own[q]) + int64_t(yv_own[q]) * Y_ONE - Yn;
            if (An >= STATE_LIMIT || An <= -STATE_LIMIT) ovf = 1;
            const int64_t Ac = An > STATE_LIMIT ? STATE_LIMIT : (An < -STATE_LIMIT ? -STATE_LIMIT : An);
            if (!skip) st_at(Aout, cc_own[q] << 2, int32_t(Ac));
            const int32_t rr = yv_own[q] * Y_ONE - int32_t(Yc);   // |rr| < 2^23: one 32 x 32 -> 64-bit product
            r2[q] = (unsigned long long)(int64_t(rr) * int64_t(rr));
        }
    }
    // residual slots.  When all lanes of a wavefront share an owner block, the MAXC sums over the wavefront are
    // taken through LDS: lanes write their MAXC residuals by copy index, then each group of G = 64 / MAXC lanes
    // sums one copy index (MAXC values per lane, then log2 G shuffle steps).  Otherwise every lane adds its
    // residuals to the slots with LDS atomics.
    {
        const int nbx = AX.nb, nbxy = AX.nb * AY.nb;
        // r_k of the block holding copy q of a pixel whose owner block is kown
        auto add_res = [&](int kown, int q, unsigned long long v) {
            const int rel = kown - kfirst;
            if (rel < CONS_SPAN) {
                atomicAdd(&s_res[rel * MAXC + q], v);
            } else if (!skip) {
                const int kq = kown - (q & 1) - ((q >> 1) & 1) * nbx - (q >> 2) * nbxy;
                atomicAdd((unsigned long long *)gp(im.resid + kq), v);
            }
        };
        const int k0 = __shfl(kk, 0);
        const bool same = __all(kk == k0);
        const int lane = tid & 63, wv = tid >> 6;
        if (same) {
            constexpr int G = 64 / MAXC;
DOPE_UNROLL
            for (int q = 0; q < MAXC; ++q) s_tr[wv][q][lane] = r2[q];
            __builtin_amdgcn_wave_barrier();
            const int q = lane / G, part = lane % G;
            unsigned long long v = 0;
DOPE_UNROLL
            for (int i = 0; i < MAXC; ++i) v += s_tr[wv][q][part * MAXC + i];
DOPE_UNROLL
            for (int sft = G / 2; sft >= 1; sft >>= 1) v += __shfl_xor(v, sft);
            if (part == 0 && v) add_res(k0, q, v);
        } else {
DOPE_UNROLL
            for (int q = 0; q < MAXC; ++q)
                if (r2[q]) add_res(kk, q, r2[q]);
        }
    }
    if (ovf) s_ovf = 1;
    __syncthreads();
    if (skip) return;   // uniform
    {
        const int klast = (chunk + 1 < im.n_chunks) ? gp(im.chunk_k0)[chunk + 1] : g.K - 1;
        const int span = min(klast - kfirst + 1, CONS_SPAN) * MAXC;
        const int nbx = AX.nb, nbxy = AX.nb * AY.nb;
        for (int b = tid; b < span; b += CONS_NT) {
            if (!s_res[b]) continue;
            const int q = b % MAXC;
            const int kq = kfirst + b / MAXC - (q & 1) - ((q >> 1) & 1) * nbx - (q >> 2) * nbxy;
            atomicAdd((unsigned long long *)gp(im.resid + kq), s_res[b]);
        }
    }
    if (tid == 0 && s_ovf) atomicOr((int32_t *)gp(&im.ctl->ovf_pending), 1);
}

// One workgroup per 256-pixel chunk of the boundary list (chunks of all images of a batch).  Chunks have even
// work, so XCD j takes a contiguous range of them (neighbouring chunks share halo lines in its L2).
template <int CONN>
__global__ __launch_bounds__(CONS_NT) void k_consensus(const Img *__restrict__ imgs, const Item *__restrict__ items) {
    const Item wi = items[xcd_item(blockIdx.x, gridDim.x)];
    consensus_chunk<CONN>(imgs[wi.img], wi.idx, -1, false);
}

// One-image consensus: descriptor and multiplier parity as kernel arguments.
template <int CONN>
__global__ __launch_bounds__(CONS_NT) void k_consensus_one(const Img one, int32_t par) {
    consensus_chunk<CONN>(one, xcd_item(blockIdx.x, gridDim.x), par, true);
}

// Loop control after the consensus of one iteration (a single workgroup): max_k r_k, stopping rule, overflow
// and solver errors, mu <- mu * mu_fact, t <- t + 1.  A separate launch instead of a last-workgroup handshake
// inside k_consensus: a device-scope fence per workgroup costs L2 write-backs on every XCD.
// Copies the loop control into the host-visible mirror (thread 0 after its own updates, so it reads them back),
// then, with system-scope release, the readback number seq into its last word: the host polls that word and
// finds the rest complete once it matches.
__device__ __forceinline__ void mirror_ctl(const GLOBAL Ctl *ctl, Ctl *mirror, int64_t seq) {
    static_assert(sizeof(Ctl) % 8 == 0 && offsetof(Ctl, seq) == sizeof(Ctl) - 8,
                  "the loop control is copied in 8-byte words, the readback number last");
    const GLOBAL unsigned long long *src = reinterpret_cast<const GLOBAL unsigned long long *>(ctl);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(mirror);
DOPE_UNROLL
    for (int i = 0; i < int(sizeof(Ctl) / 8) - 1; ++i) dst[i] = src[i];
    // release at system scope: the words above reach host memory first (written back from the L2 if the mirror
    // is cached there), then this store, which goes through at system scope
    __hip_atomic_store(&mirror->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// mirror (single-image launches only): host-visible copy of the loop control to refresh after the update.
__device__ __forceinline__ void finalize_image(const Img &im, Ctl *mirror = nullptr, int64_t seq = 0) {
    GLOBAL Ctl *ctl = gp(im.ctl);
    // every load is issued before any is used (one memory round trip): the loop control and the residuals
    const int32_t halted = ctl->halted, t = ctl->t, t_limit = ctl->t_limit, solver_err = ctl->solver_err,
                  ovf = ctl->ovf_pending, stop_conv = ctl->stop_on_converge, mu_num = ctl->mu_num,
                  mu_den = ctl->mu_den, status = ctl->status, vpending = ctl->vpending, flags = ctl->flags,
                  allow_negative = ctl->allow_negative;
    const int64_t M = ctl->M;
    const uint64_t eps2 = ctl->eps2;
    __shared__ unsigned long long s_max[4];
    const int tid = threadIdx.x;
    const int K = im.g.K;
    const GLOBAL int64_t *resid = gp(im.resid);
    // the first two residuals of this thread (clamped indices, masked afterwards), then any others
    const uint64_t v0 = static_cast<uint64_t>(resid[tid < K ? tid : 0]);
    const uint64_t v1 = static_cast<uint64_t>(resid[tid + 256 < K ? tid + 256 : 0]);
    unsigned long long mx = tid < K ? v0 : 0;
    if (tid + 256 < K && v1 > mx) mx = v1;
    for (int k = tid + 512; k < K; k += 256) {
        const unsigned long long v = static_cast<unsigned long long>(resid[k]);
        mx = v > mx ? v : mx;
    }
    // a verdict still pending (a solve straight after the energy upload): taken here; a rejected energy halts the
    // loop with t unchanged (the iteration kernels skipped it)
    const int32_t vst = vpending ? energy_verdict(flags, allow_negative) : 0;
    if (vpending && tid == 0) {
        ctl->vflags = flags;
        ctl->flags = 0;
        ctl->vpending = 0;
        if (vst) {
            ctl->status = vst;
            ctl->halted = 1;
        }
    }
    if (halted != 0 || t >= t_limit || vst != 0) {   // uniform
        if (tid == 0) {
            if (vst && im.summary) {
                GLOBAL int32_t *sm = gp(im.summary);
                sm[0] = t;
                sm[1] = 1;
                sm[2] = 0;
                sm[3] = vst;
            }
            if (mirror) mirror_ctl(ctl, mirror, seq);
        }
        return;
    }
DOPE_UNROLL
    for (int sft = 32; sft >= 1; sft >>= 1) {
        const unsigned long long o = __shfl_xor(mx, sft);
        mx = o > mx ? o : mx;
    }
    if ((tid & 63) == 0) s_max[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        for (int wv = 0; wv < 4; ++wv) mx = s_max[wv] > mx ? s_max[wv] : mx;
        ctl->last_max_resid = mx;
        const int conv = mx <= eps2 ? 1 : 0;
        ctl->converged = conv;
        int st_new = 0, halt_new = 0;
        if (solver_err) { st_new = -6; halt_new = 1; }
        if (ovf) { st_new = -5; halt_new = 1; }
        if (stop_conv && conv) halt_new = 1;
        if (st_new) ctl->status = st_new;
        if (halt_new) ctl->halted = 1;
        const int64_t Mn = (M * mu_num) / mu_den;
        ctl->M = Mn > MU_MAX ? MU_MAX : Mn;
        ctl->t = t + 1;
        ctl->ovf_pending = 0;
        ctl->solver_err = 0;
        if (im.summary) {
            GLOBAL int32_t *sm = gp(im.summary);
            sm[0] = t + 1;
            sm[1] = halt_new;
            sm[2] = conv;
            sm[3] = st_new ? st_new : status;
        }
        if (mirror) mirror_ctl(ctl, mirror, seq);
    }
}

// One workgroup per image (one = the only image's descriptor when single != 0).
__global__ __launch_bounds__(256) void k_finalize(const Img *__restrict__ imgs, Queue *queue, const Img one,
                                                  int32_t single, Ctl *mirror, int64_t seq) {
    if (blockIdx.x == 0 && threadIdx.x == 0) queue->next = 0;   // next iteration's block-solve queue
    if (single) finalize_image(one, mirror, seq);
    else finalize_image(imgs[blockIdx.x]);
}

// ------------------------------------------------------------------------------------------------------------
// Setup, labels and energy
// ------------------------------------------------------------------------------------------------------------

// Everything set_energy puts on the device, in one launch over the pixel grid (grid: (ceil(W/256), H*D)):
//   - a copy of u into the workspace (skipped when the source already is the workspace copy; w is not kept: the
//     energy kernel recovers lambda_q8 w_ij exactly from c_ij),
//   - c_ij = lambda_q8 w_ij 64 / (q_i q_j) for the half-stencil edges of every pixel, with validation bits (nonzero
//     weight on an off-grid edge, negative weight, per-node sum_j |c_ij| >= 2^29) OR-ed into ctl->flags,
//   - the initial ADMM state (Y = 1/2, A = 0, yhat = 0, r_k = 0; a grid-stride pass over the block-major arrays),
//   - the loop control (workgroup (0, 0)), left as a solve starts it (limit si.t_limit, halting when the stopping
//     rule holds) with the validation verdict pending; ctl->flags is left alone: the verdict consumes and clears
//     it.  The verdict is taken by the next control kernel (the first iteration's k_finalize included), and until
//     then the iteration kernels skip an energy that fails it (ctl_skip).
struct StateInit {
    int64_t mu0;
    uint64_t eps2;
    int32_t mu_num, mu_den;
    int32_t allow_negative;
    int32_t t_limit;   // iteration limit a solve runs under
};

// Returns the validation bits (FLAG_*) of the pixel's weights.
template <int CONN>
__device__ __forceinline__ int setup_pixel(const Geom &g, int gx, int gy, int gz, const int32_t *__restrict__ u_src,
                                           const int32_t *__restrict__ w_src, int32_t *__restrict__ u_ws,
                                           int32_t *__restrict__ cw, int32_t lam, int32_t *__restrict__ Y) {
    constexpr int H = Sten<CONN>::H;
    constexpr int ND = 2 * H;
    const uint32_t i = uint32_t(gx) + uint32_t(g.W) * (uint32_t(gy) + uint32_t(g.H) * uint32_t(gz));
    const uint32_t bi = i << 2;
    BoxCov<CONN> bc;
    bc.init(g, gx, gy, gz);
    const int lqi = bc.lq(make_int3(0, 0, 0));   // log2 q of this pixel
    const DirMask<CONN> ing = inside_mask<CONN>(gx, gy, gz, g.W, g.H, g.D);
    // all loads first (an off-grid neighbour reads pixel i itself and is masked); the edge's weight lives at the
    // pixel holding its positive half-edge
    const GLOBAL int32_t *wg = gp(w_src);
    int32_t ui = ld_at(gp(u_src), bi);
    int32_t wl[ND];
DOPE_UNROLL
    for (int d = 0; d < ND; ++d) {
        const int3 v = full_dir<CONN>(d);
        const int32_t dl = v.x + g.W * (v.y + g.H * v.z);
        uint32_t bj = (d >= H && ((ing >> d) & 1u)) ? bi + (uint32_t(dl) << 2) : bi;
        asm("" : "+v"(bj));   // optimisation barrier only: keeps the loads unconditional
        wl[d] = ld_at(wg + int64_t(d < H ? d : d - H) * g.n, bj);
    }
    int flags = 0;
    int64_t sum = 0;
DOPE_UNROLL
    for (int d = 0; d < ND; ++d) {
        const int3 v = full_dir<CONN>(d);
        const bool on = (ing >> d) & 1u;
        const int32_t wv = (d < H || on) ? wl[d] : 0;
        const int lqj = bc.lq(v);
        // c = lambda_q8 w 64 / (q_i q_j): q_i q_j = 2^(lqi + lqj) <= 64 (0 for an off-grid neighbour)
        const int64_t cvv = on ? int64_t(lam) * int64_t(wv) * (int64_t(1) << (6 - lqi - lqj)) : 0;
        const bool big = cvv >= CAP_SUM_LIMIT || cvv <= -CAP_SUM_LIMIT;
        flags |= (!on && wv != 0) ? FLAG_OFFGRID : 0;
        flags |= (on && wv < 0) ? FLAG_NEGATIVE : 0;
        flags |= big ? FLAG_TOOBIG : 0;
        sum += cvv < 0 ? -cvv : cvv;
        if (d < H) st_at(gp(cw) + int64_t(d) * g.n, bi, big ? 0 : int32_t(cvv));
    }
    if (u_src != u_ws) st_at(gp(u_ws), bi, ui);
    st_at(gp(Y), bi, int32_t(Y_HALF));
    if (sum >= CAP_SUM_LIMIT) flags |= FLAG_TOOBIG;
    return flags;
}


template <int CONN>
__global__ __launch_bounds__(256) void k_setup(Geom g, const int32_t *__restrict__ u_src,
                                               const int32_t *__restrict__ w_src, int32_t *__restrict__ u_ws,
                                               int32_t *__restrict__ cw, int32_t lam,
                                               int32_t *__restrict__ Y, int32_t *__restrict__ A0,
                                               int32_t *__restrict__ A1, uint8_t *__restrict__ yhat,
                                               int64_t *__restrict__ resid, Ctl *ctl, StateInit si) {
    // block-major arrays and the loop control
    {
        const int64_t T = int64_t(gridDim.x) * gridDim.y * 256;
        const int64_t t0 = (int64_t(blockIdx.y) * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
        for (uint32_t i = uint32_t(t0); i < uint32_t(g.tot); i += uint32_t(T)) {   // copies < 2^30
            st_at(gp(A0), i << 2, int32_t(0));
            st_at(gp(A1), i << 2, int32_t(0));
            st_at(gp(yhat), i, uint8_t(0));
        }
        for (int64_t i = t0; i < g.K; i += T) resid[i] = 0;
        if (t0 == 0) {
            GLOBAL Ctl *c = gp(ctl);
            c->M = si.mu0;
            c->max_resid = 0;
            c->last_max_resid = 0;
            c->eps2 = si.eps2;
            c->energy = 0;
            c->t = 0;
            c->t_limit = si.t_limit;
            c->stop_on_converge = 1;
            c->converged = 0;
            c->halted = 0;
            c->status = 0;
            c->ovf_pending = 0;
            c->solver_err = 0;
            c->wg_counter = 0;
            c->mu_num = si.mu_num;
            c->mu_den = si.mu_den;
            c->vflags = 0;
            c->vpending = 1;
            c->allow_negative = si.allow_negative;
        }
    }
    const int gx = blockIdx.x * 256 + threadIdx.x;
    if (gx >= g.W) return;
    const int rows = g.H * g.D;
    int flags = 0;
    for (int row = blockIdx.y; row < rows; row += gridDim.y)
        flags |= setup_pixel<CONN>(g, gx, row % g.H, row / g.H, u_src, w_src, u_ws, cw, lam, Y);
    if (flags) atomicOr((int32_t *)gp(&ctl->flags), flags);
}

// Batched energy upload: workgroup b sets up pixel row rows[b].idx of image rows[b].img (row = y + H z) and its
// share of the image's block-major arrays; the image's row 0 also resets its loop control.
template <int CONN>
__global__ __launch_bounds__(256) void k_setup_batch(const Img *__restrict__ imgs, const SetupArg *__restrict__ args,
                                                     const Item *__restrict__ rows) {
    const Item wi = rows[blockIdx.x];
    const Img &im = const_img(imgs + wi.img);
    const SetupArg &a = args[wi.img];
    const Geom &g = im.g;
    const int nrows = g.H * g.D;
    const int row = wi.idx;
    {
        const int64_t lo = g.tot * row / nrows, hi = g.tot * (row + 1) / nrows;
        for (uint32_t i = uint32_t(lo) + threadIdx.x; i < uint32_t(hi); i += 256) {   // copies < 2^30
            st_at(gp(im.A0), i << 2, int32_t(0));
            st_at(gp(im.A1), i << 2, int32_t(0));
            st_at(gp(im.yhat), i, uint8_t(0));
        }
        const int64_t klo = int64_t(g.K) * row / nrows, khi = int64_t(g.K) * (row + 1) / nrows;
        for (int64_t k = klo + threadIdx.x; k < khi; k += 256) gp(im.resid)[k] = 0;
        if (row == 0 && threadIdx.x == 0) {
            GLOBAL Ctl *c = gp(im.ctl);
            c->M = a.mu0;
            c->max_resid = 0;
            c->last_max_resid = 0;
            c->eps2 = a.eps2;
            c->energy = 0;
            c->t = 0;
            c->t_limit = 0;
            c->stop_on_converge = 0;
            c->converged = 0;
            c->halted = 0;
            c->status = 0;
            c->ovf_pending = 0;
            c->solver_err = 0;
            c->wg_counter = 0;
            c->mu_num = a.mu_num;
            c->mu_den = a.mu_den;
            c->vflags = 0;
            c->vpending = 1;
            c->allow_negative = a.allow_negative;
        }
    }
    int flags = 0;
    for (int gx = threadIdx.x; gx < g.W; gx += 256)
        flags |= setup_pixel<CONN>(g, gx, row % g.H, row / g.H, a.u_src, a.w_src, const_cast<int32_t *>(im.u),
                                   const_cast<int32_t *>(im.cw), a.lam_q8, im.Y);
    if (flags) atomicOr((int32_t *)gp(&im.ctl->flags), flags);
}

// Batched labels: workgroup b writes pixel row rows[b].idx of image rows[b].img into labels[img].
__global__ __launch_bounds__(256) void k_labels_batch(const Img *__restrict__ imgs, uint8_t *const *__restrict__ labels,
                                                      const Item *__restrict__ rows) {
    const Item wi = rows[blockIdx.x];
    const Img &im = const_img(imgs + wi.img);
    const GLOBAL int32_t *Y = gp(im.Y);
    GLOBAL uint8_t *out = gp(labels[wi.img]);
    const int64_t base = int64_t(im.g.W) * wi.idx;
    for (int gx = threadIdx.x; gx < im.g.W; gx += 256) out[base + gx] = uint8_t(Y[base + gx] > Y_HALF);
}

// Energy validation verdict of a pending set-up: off-grid or oversized weights -> EINVAL; a negative weight
// when the resolved solver is max-flow -> ENOTSUBMODULAR.  Stops the loop before any iteration runs.  The
// accumulated bits move to ctl->vflags (read by the host for the error message) and the accumulator is cleared
// for the next setup.  Runs in the single thread of a control kernel.
__device__ __forceinline__ void validate_pending(Ctl *ctl) {
    GLOBAL Ctl *c = gp(ctl);
    if (!c->vpending) return;
    const int32_t f = c->flags;
    c->vflags = f;
    c->flags = 0;
    c->vpending = 0;
    int32_t st = 0;
    if (f & (FLAG_OFFGRID | FLAG_TOOBIG)) st = -1;
    else if ((f & FLAG_NEGATIVE) && !c->allow_negative) st = -4;
    if (st) {
        c->status = st;
        c->halted = 1;
    }
}

__global__ void k_validate(Ctl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) validate_pending(ctl);
}

__global__ void k_batch_setup(const Img *__restrict__ imgs, int32_t n, const int32_t *__restrict__ params) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    GLOBAL Ctl *ctl = gp(imgs[i].ctl);
    validate_pending(imgs[i].ctl);
    ctl->t_limit = params[2 * i];
    ctl->stop_on_converge = params[2 * i + 1];
    if (ctl->status == 0) ctl->halted = 0;
    // the summary also reports images that will not run (an energy that failed validation)
    if (imgs[i].summary) {
        GLOBAL int32_t *sm = gp(imgs[i].summary);
        sm[0] = ctl->t;
        sm[1] = ctl->halted;
        sm[2] = ctl->converged;
        sm[3] = ctl->status;
    }
}

// Same effect as validate_pending followed by the loop-limit update, with every field loaded in one round trip.
__global__ void k_ctl_setup(Ctl *ctl, int32_t t_limit, int32_t stop_on_converge, int32_t clear_energy) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        GLOBAL Ctl *c = gp(ctl);
        const int32_t vpending = c->vpending, f = c->flags, allow_negative = c->allow_negative,
                      status = c->status;
        int32_t st = 0;
        if (vpending) {
            c->vflags = f;
            c->flags = 0;
            c->vpending = 0;
            if (f & (FLAG_OFFGRID | FLAG_TOOBIG)) st = -1;
            else if ((f & FLAG_NEGATIVE) && !allow_negative) st = -4;
            if (st) c->status = st;
        }
        c->t_limit = t_limit;
        c->stop_on_converge = stop_on_converge;
        if (st) c->halted = 1;
        else if (status == 0) c->halted = 0;
        if (clear_energy) c->energy = 0;
    }
}

// Labels [Y > 2^15].  grid: (ceil(W/256), rows), rows strided over H*D.
__global__ __launch_bounds__(256) void k_labels(Geom g, const int32_t *__restrict__ Y, uint8_t *__restrict__ labels) {
    const int gx = blockIdx.x * 256 + threadIdx.x;
    if (gx >= g.W) return;
    const int rows = g.H * g.D;
    for (int row = blockIdx.y; row < rows; row += gridDim.y) {
        const int64_t i = int64_t(gx) + int64_t(g.W) * row;
        labels[i] = uint8_t(Y[i] > Y_HALF);
    }
}

constexpr int ENERGY_WGS = 256;

// Per-workgroup partial sums of E_q = 256 u.l + lambda_q8 sum_edges w |l_i - l_j| (grid-stride over pixels,
// ENERGY_WGS workgroups, no atomics); k_energy_sum adds the partials into ctl->energy.
template <int CONN>
__global__ __launch_bounds__(256) void k_energy(Geom g, const int32_t *__restrict__ u, const int32_t *__restrict__ cw,
                                                const int32_t *__restrict__ Y, int64_t *__restrict__ part) {
    constexpr int H = Sten<CONN>::H;
    __shared__ long long s_sum[4];
    long long e = 0;
    const int64_t rows = int64_t(g.H) * g.D;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int gy = int(row % g.H), gz = int(row / g.H);
        for (int gx = threadIdx.x; gx < g.W; gx += 256) {
            const int64_t i = lin(g, gx, gy, gz);
            const int li = Y[i] > Y_HALF;
            if (li) e += 256ll * u[i];
            BoxCov<CONN> bc;
            bc.init(g, gx, gy, gz);
            const int lqi = bc.lq(make_int3(0, 0, 0));
DOPE_UNROLL
            for (int o = 0; o < H; ++o) {
                const int3 v = half_off<CONN>(o);
                if (!in_grid(g, gx + v.x, gy + v.y, gz + v.z)) continue;
                const int lj = Y[lin(g, gx + v.x, gy + v.y, gz + v.z)] > Y_HALF;
                if (li == lj) continue;
                // lambda_q8 w_ij = c_ij q_i q_j / 64 exactly (c_ij = lambda_q8 w_ij 64 / (q_i q_j), q a power of two)
                const int lqj = bc.lq(v);
                e += (static_cast<long long>(cw[int64_t(o) * g.n + i]) << (lqi + lqj)) >> 6;
            }
        }
    }
DOPE_UNROLL
    for (int sft = 32; sft >= 1; sft >>= 1) e += __shfl_xor(e, sft);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
}

__global__ __launch_bounds__(256) void k_energy_sum(const int64_t *__restrict__ part, int n, Ctl *ctl) {
    __shared__ long long s_sum[4];
    long long e = 0;
    for (int i = threadIdx.x; i < n; i += 256) e += part[i];
DOPE_UNROLL
    for (int sft = 32; sft >= 1; sft >>= 1) e += __shfl_xor(e, sft);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) ctl->energy = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
}

inline unsigned blocks_for(int64_t n, int nt) { return unsigned((n + nt - 1) / nt); }
// Grid rows of the pixel kernels: one per image row up to the grid's y limit; kernels stride over the rest.
inline unsigned row_blocks(const Geom &g) {
    const int64_t rows = int64_t(g.H) * g.D;
    return unsigned(rows < 65535 ? rows : 65535);
}

template <int CONN, int NT>
hipError_t launch_maxflow(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    constexpr int H = Sten<CONN>::H;
    const size_t lds = maxflow_lds_bytes(grp.npmax, H);
    // The dynamic-LDS limit of these kernels is raised once per process to the whole 160 KiB (every block the
    // host admits fits it), so launches from contexts on several threads never race on the attribute.
    static std::once_flag lds_once;
    static hipError_t lds_err = hipSuccess;
    std::call_once(lds_once, [] {
        const void *fns[3] = {reinterpret_cast<const void *>(&k_block_solve<CONN, NT>),
                              reinterpret_cast<const void *>(&k_block_solve_queue<CONN, NT>),
                              reinterpret_cast<const void *>(&k_block_solve_one<CONN, NT>)};
        for (const void *f : fns)
            if (lds_err == hipSuccess)
                lds_err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(MAXFLOW_LDS_LIMIT));
    });
    if (lds_err != hipSuccess) return lds_err;
    if (lds > MAXFLOW_LDS_LIMIT) return hipErrorInvalidValue;
    if ((grp.npmax + NT - 1) / NT > 16) return hipErrorInvalidValue;   // the residual lane sums assume <= 16
    const int32_t round_limit = 65536 + 64 * grp.npmax;
    const int32_t workers = grp.n_workers > 0 ? (grp.n_workers < grp.n_blk_items ? grp.n_workers : grp.n_blk_items)
                                              : grp.n_blk_items;
    const int32_t direct = workers == grp.n_blk_items ? 1 : 0;
    const int32_t relabel_period = grp.npmax > 2048 ? 8 : 4;
    // the events carry the dispatch's own start and end timestamps (no marker packets around the launch)
    if (grp.one && direct) {
        if (e0) hipExtLaunchKernelGGL(k_block_solve_one<CONN, NT>, dim3(workers), dim3(NT), uint32_t(lds), s, e0, e1,
                                      0u, *grp.one, grp.par, grp.npmax, round_limit, relabel_period);
        else hipLaunchKernelGGL((k_block_solve_one<CONN, NT>), dim3(workers), dim3(NT), lds, s, *grp.one, grp.par,
                                grp.npmax, round_limit, relabel_period);
    } else if (direct) {
        if (e0) hipExtLaunchKernelGGL(k_block_solve<CONN, NT>, dim3(workers), dim3(NT), uint32_t(lds), s, e0, e1, 0u,
                                      grp.imgs, grp.blk_items, grp.npmax, round_limit, relabel_period);
        else hipLaunchKernelGGL((k_block_solve<CONN, NT>), dim3(workers), dim3(NT), lds, s, grp.imgs, grp.blk_items,
                                grp.npmax, round_limit, relabel_period);
    } else {
        if (e0) hipExtLaunchKernelGGL(k_block_solve_queue<CONN, NT>, dim3(workers), dim3(NT), uint32_t(lds), s, e0, e1,
                                      0u, grp.imgs, grp.blk_items, grp.n_blk_items, grp.queue, grp.npmax, round_limit,
                                      relabel_period);
        else hipLaunchKernelGGL((k_block_solve_queue<CONN, NT>), dim3(workers), dim3(NT), lds, s, grp.imgs,
                                grp.blk_items, grp.n_blk_items, grp.queue, grp.npmax, round_limit, relabel_period);
    }
    return hipGetLastError();
}

// Slices per block of k_block_prep_gmem: at most PREP_SLICE_MAX nodes each, and as many as fill the last round of
// workgroups best (one 1024-thread workgroup per CU at a time): 128 blocks of 11340 nodes take 4 slices (two full
// rounds) rather than 3 (a round and a half).
inline int32_t prep_slices(int32_t npmax, int32_t nb) {
    const int32_t lo = (npmax + PREP_SLICE_MAX - 1) / PREP_SLICE_MAX;
    int32_t best = lo;
    double best_fill = 0.0;
    for (int32_t n = lo; n <= PREP_SLICES_MAX; ++n) {
        const int64_t wgs = int64_t(nb) * n;
        const double fill = double(wgs) / double(((wgs + NUM_CUS - 1) / NUM_CUS) * NUM_CUS);
        if (fill > best_fill + 1e-9) {
            best = n;
            best_fill = fill;
        }
    }
    return best;
}

template <int CONN>
hipError_t launch_maxflow_gmem(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    constexpr int NT = gmem_threads(CONN);
    if (!grp.one || grp.npmax > gmem_max_np(CONN) || grp.gstride < maxflow_lds_bytes(grp.npmax, Sten<CONN>::H))
        return hipErrorInvalidValue;
    const int32_t round_limit = 65536 + 64 * grp.npmax;
    const int32_t relabel_period = 8;
    const dim3 grid(unsigned(grp.n_blk_items));
    // the per-node arrays go to LDS when they fit there (the edge arrays are 8h of every node's 8h + 9 + m bytes)
    static std::once_flag lds_once;
    static hipError_t lds_err = hipSuccess;
    std::call_once(lds_once, [] {
        lds_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_block_solve_gmem<CONN, NT>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(MAXFLOW_LDS_LIMIT));
    });
    if (lds_err != hipSuccess) return lds_err;
    const size_t node_lds = maxflow_node_lds_bytes(grp.npmax, Sten<CONN>::H);
    const int32_t split = node_lds <= MAXFLOW_LDS_LIMIT ? 1 : 0;
    const uint32_t lds = split ? uint32_t(node_lds) : 0u;
    if constexpr (2 * Sten<CONN>::H <= 8) {
        if (split && grp.npmax > PREP_MIN_NP) {
            // two launches: slices of every block's prologue and elimination on several CUs, then the rest
            static std::once_flag flow_once;
            static hipError_t flow_err = hipSuccess;
            std::call_once(flow_once, [] {
                flow_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_block_flow_gmem<CONN, NT>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(MAXFLOW_LDS_LIMIT));
            });
            if (flow_err != hipSuccess) return flow_err;
            const int32_t nb = grp.n_blk_items;
            const int32_t nslice = prep_slices(grp.npmax, nb);
            if (nslice < 1 || nslice > PREP_SLICES_MAX || (grp.npmax + nslice - 1) / nslice > PREP_SLICE_MAX)
                return hipErrorInvalidValue;
            const uint32_t plds = uint32_t(64 + 7 * PREP_SLICE_MAX);
            const dim3 pgrid(unsigned(nb) * unsigned(nslice));
            if (e0) {
                hipExtLaunchKernelGGL(k_block_prep_gmem<CONN, NT>, pgrid, dim3(NT), plds, s, e0, nullptr, 0u,
                                      *grp.one, grp.par, grp.npmax, grp.gscratch, grp.gstride, nb, nslice);
                hipExtLaunchKernelGGL(k_block_flow_gmem<CONN, NT>, grid, dim3(NT), lds, s, nullptr, e1, 0u,
                                      *grp.one, grp.par, grp.npmax, round_limit, relabel_period, grp.gscratch,
                                      grp.gstride);
            } else {
                hipLaunchKernelGGL((k_block_prep_gmem<CONN, NT>), pgrid, dim3(NT), plds, s, *grp.one, grp.par,
                                   grp.npmax, grp.gscratch, grp.gstride, nb, nslice);
                hipLaunchKernelGGL((k_block_flow_gmem<CONN, NT>), grid, dim3(NT), lds, s, *grp.one, grp.par,
                                   grp.npmax, round_limit, relabel_period, grp.gscratch, grp.gstride);
            }
            return hipGetLastError();
        }
    }
    if (e0) hipExtLaunchKernelGGL(k_block_solve_gmem<CONN, NT>, grid, dim3(NT), lds, s, e0, e1, 0u, *grp.one, grp.par,
                                  grp.npmax, round_limit, relabel_period, grp.gscratch, grp.gstride, split);
    else hipLaunchKernelGGL((k_block_solve_gmem<CONN, NT>), grid, dim3(NT), lds, s, *grp.one, grp.par, grp.npmax,
                            round_limit, relabel_period, grp.gscratch, grp.gstride, split);
    return hipGetLastError();
}

template <int CONN>
hipError_t launch_lsatr(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (dir_mask_bytes(Sten<CONN>::H) == 1) {
        const size_t lds = lsatr_lds_bytes(grp.npmax, Sten<CONN>::H);
        static std::once_flag lds_once;
        static hipError_t lds_err = hipSuccess;
        std::call_once(lds_once, [] {
            lds_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_block_lsatr<CONN>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(LDS_LIMIT - 64));
        });
        if (lds_err != hipSuccess) return lds_err;
        if (lds > LDS_LIMIT - 64 || grp.npmax > LSATR_MAX_NP) return hipErrorInvalidValue;
        const int32_t round_limit = 65536 + 64 * grp.npmax;
        const int32_t relabel_period = 4;
        const dim3 grid(unsigned(grp.n_blk_items));
        if (e0) hipExtLaunchKernelGGL(k_block_lsatr<CONN>, grid, dim3(LSATR_THREADS), uint32_t(lds), s, e0, e1, 0u,
                                      grp.imgs, grp.blk_items, grp.npmax, round_limit, relabel_period);
        else hipLaunchKernelGGL(k_block_lsatr<CONN>, grid, dim3(LSATR_THREADS), lds, s, grp.imgs, grp.blk_items,
                                grp.npmax, round_limit, relabel_period);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int CONN>
hipError_t solve_phase(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (grp.solver == 3) return launch_lsatr<CONN>(grp, s, e0, e1);
    if (grp.solver == 2) {
        if (e0) {
            hipExtLaunchKernelGGL(k_block_exhaustive<CONN>, dim3(blocks_for(grp.n_blk_items, EX_WAVES)), dim3(256),
                                  0u, s, e0, e1, 0u, grp.imgs, grp.blk_items, grp.n_blk_items);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_block_exhaustive<CONN>, dim3(blocks_for(grp.n_blk_items, EX_WAVES)), dim3(256), 0, s,
                           grp.imgs, grp.blk_items, grp.n_blk_items);
        return hipGetLastError();
    }
    if (grp.gscratch) return launch_maxflow_gmem<CONN>(grp, s, e0, e1);   // blocks beyond the LDS
    // Workgroup size: blocks of more than 512 pixels use 1024 threads when every block gets a CU of its own
    // (or when the LDS footprint allows only one block per CU), otherwise 512 threads so that all blocks are
    // resident at once and neighbours on a CU hide each other's barrier and LDS latency.  Measured on MI355X with
    // 32x32 8-connected blocks: 289 and 1089 blocks both favour 512 threads.
    // stencils so wide that no block of more than 512 pixels fits the LDS get the 256-thread kernels only
    if constexpr (maxflow_lds_bytes(513, Sten<CONN>::H) > MAXFLOW_LDS_LIMIT) {
        return launch_maxflow<CONN, 256>(grp, s, e0, e1);
    } else {
        if (grp.npmax > 512) {
            const bool one_per_cu = maxflow_lds_bytes(grp.npmax, Sten<CONN>::H) > MAXFLOW_LDS_LIMIT / 2;
            if (one_per_cu || grp.n_blk_items <= NUM_CUS) return launch_maxflow<CONN, 1024>(grp, s, e0, e1);
            return launch_maxflow<CONN, 512>(grp, s, e0, e1);
        }
        return launch_maxflow<CONN, 256>(grp, s, e0, e1);
    }
}

template <int CONN>
void consensus_launch(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid(unsigned(grp.n_chk_items));
    if (grp.one) {
        if (e0) hipExtLaunchKernelGGL(k_consensus_one<CONN>, grid, dim3(CONS_NT), 0u, s, e0, e1, 0u, *grp.one, grp.par);
        else hipLaunchKernelGGL(k_consensus_one<CONN>, grid, dim3(CONS_NT), 0, s, *grp.one, grp.par);
    } else {
        if (e0) hipExtLaunchKernelGGL(k_consensus<CONN>, grid, dim3(CONS_NT), 0u, s, e0, e1, 0u, grp.imgs,
                                      grp.chk_items);
        else hipLaunchKernelGGL(k_consensus<CONN>, grid, dim3(CONS_NT), 0, s, grp.imgs, grp.chk_items);
    }
}

}  // namespace

// Per-stencil entry points.  Each stencil's kernels are compiled in a translation unit of their own (this file
// with DOPE_CONN defined, see the build script), which instantiates these; the launchers below dispatch on the
// stencil at run time.
template <int CONN>
hipError_t conn_setup(const Geom &g, const int32_t *u_src, const int32_t *w_src, int32_t *u_ws, int32_t *cw,
                      int32_t lam_q8, int32_t *Y, int32_t *A0, int32_t *A1, uint8_t *yhat, int64_t *resid, Ctl *ctl,
                      int64_t mu0, uint64_t eps2, int32_t mu_num, int32_t mu_den, int32_t allow_negative,
                      int32_t t_limit, hipStream_t s) {
    const StateInit si{mu0, eps2, mu_num, mu_den, allow_negative, t_limit};
    hipLaunchKernelGGL(k_setup<CONN>, dim3(blocks_for(g.W, 256), row_blocks(g)), dim3(256), 0, s, g, u_src, w_src,
                       u_ws, cw, lam_q8, Y, A0, A1, yhat, resid, ctl, si);
    return hipGetLastError();
}

template <int CONN>
hipError_t conn_setup_batch(const Img *imgs, const SetupArg *args, const Item *rows, int32_t n_rows, hipStream_t s) {
    hipLaunchKernelGGL(k_setup_batch<CONN>, dim3(unsigned(n_rows)), dim3(256), 0, s, imgs, args, rows);
    return hipGetLastError();
}

template <int CONN>
hipError_t conn_solve(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return solve_phase<CONN>(grp, s, e0, e1);
}

template <int CONN>
hipError_t conn_consensus(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    consensus_launch<CONN>(grp, s, e0, e1);
    return hipGetLastError();
}

template <int CONN>
hipError_t conn_energy(const Geom &g, const int32_t *u, const int32_t *cw, const int32_t *Y, int64_t *part,
                       unsigned wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_energy<CONN>, dim3(wgs), dim3(256), 0, s, g, u, cw, Y, part);
    return hipGetLastError();
}

#define DOPE_CONN_ENTRIES(SPEC, C)                                                                                 \
    SPEC template hipError_t conn_setup<C>(const Geom &, const int32_t *, const int32_t *, int32_t *, int32_t *,    \
                                           int32_t, int32_t *, int32_t *, int32_t *, uint8_t *, int64_t *, Ctl *,   \
                                           int64_t, uint64_t, int32_t, int32_t, int32_t, int32_t, hipStream_t);     \
    SPEC template hipError_t conn_setup_batch<C>(const Img *, const SetupArg *, const Item *, int32_t, hipStream_t); \
    SPEC template hipError_t conn_solve<C>(const Group &, hipStream_t, hipEvent_t, hipEvent_t);                      \
    SPEC template hipError_t conn_consensus<C>(const Group &, hipStream_t, hipEvent_t, hipEvent_t);                  \
    SPEC template hipError_t conn_energy<C>(const Geom &, const int32_t *, const int32_t *, const int32_t *,         \
                                            int64_t *, unsigned, hipStream_t);

#ifdef DOPE_CONN
DOPE_CONN_ENTRIES(, DOPE_CONN)
#else
// instantiated by the per-stencil translation units
DOPE_CONN_ENTRIES(extern, 4)
DOPE_CONN_ENTRIES(extern, 8)
DOPE_CONN_ENTRIES(extern, 24)
DOPE_CONN_ENTRIES(extern, 48)
DOPE_CONN_ENTRIES(extern, 80)
DOPE_CONN_ENTRIES(extern, 6)
DOPE_CONN_ENTRIES(extern, 32)
DOPE_CONN_ENTRIES(extern, 122)
DOPE_CONN_ENTRIES(extern, 256)

// Run-time dispatch on the stencil; f is called as f(std::integral_constant<int, CONN>()).
template <class F>
hipError_t by_conn(int32_t conn, F &&f) {
    switch (conn) {
        case 4: return f(std::integral_constant<int, 4>());
        case 8: return f(std::integral_constant<int, 8>());
        case 24: return f(std::integral_constant<int, 24>());
        case 48: return f(std::integral_constant<int, 48>());
        case 80: return f(std::integral_constant<int, 80>());
        case 6: return f(std::integral_constant<int, 6>());
        case 32: return f(std::integral_constant<int, 32>());
        case 122: return f(std::integral_constant<int, 122>());
        case 256: return f(std::integral_constant<int, 256>());
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_setup(const Geom &g, const int32_t *u_src, const int32_t *w_src, int32_t *u_ws, int32_t *cw,
                        int32_t lam_q8, int32_t *Y, int32_t *A0, int32_t *A1, uint8_t *yhat,
                        int64_t *resid, Ctl *ctl, int64_t mu0, int32_t mu_num, int32_t mu_den, uint64_t eps2,
                        int32_t allow_negative, int32_t t_limit, hipStream_t s) {
    return by_conn(g.conn, [&](auto c) {
        return conn_setup<decltype(c)::value>(g, u_src, w_src, u_ws, cw, lam_q8, Y, A0, A1, yhat, resid, ctl, mu0,
                                              eps2, mu_num, mu_den, allow_negative, t_limit, s);
    });
}

// One workgroup per block: the owner copies of the block's pixels that are not interior to it, in the block's
// local raster order (the owned box is a prefix of the block along every axis), from entry btab[k][7].  Ranks come
// from wavefront ballots and a prefix over the four wavefronts of each 256-position pass.
__global__ __launch_bounds__(256) void k_build_blist(Geom g, const int32_t *__restrict__ btab,
                                                     int32_t *__restrict__ blist) {
    __shared__ int s_wc[4];
    const int k = blockIdx.x;
    const int32_t *r = btab + int64_t(BTAB_STRIDE) * k;
    const int t[3] = {k % g.ax[0].nb, (k / g.ax[0].nb) % g.ax[1].nb, k / (g.ax[0].nb * g.ax[1].nb)};
    int ol[3], lo[3], hi[3];
DOPE_UNROLL
    for (int a = 0; a < 3; ++a) {
        const Axis &ax = g.ax[a];
        const int start = t[a] * ax.s;
        ol[a] = t[a] < ax.nb - 1 ? ax.s : ax.N - start;
        lo[a] = axis_interior_lo(ax, t[a], g.rad) - start;
        hi[a] = axis_interior_hi(ax, t[a], g.rad) - start;
    }
    const int total = ol[0] * ol[1] * ol[2];
    const int ex = r[3], ey = r[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int run = r[7];
    for (int b = 0; b < total; b += 256) {
        const int i = b + tid;
        const int lx = i % ol[0], rr = i / ol[0], ly = rr % ol[1], lz = rr / ol[1];
        const bool inner = lx >= lo[0] && lx < hi[0] && ly >= lo[1] && ly < hi[1] && lz >= lo[2] && lz < hi[2];
        const bool flag = i < total && !inner;
        const unsigned long long m = __ballot(flag);
        if (lane == 0) s_wc[wv] = __popcll(m);
        __syncthreads();
        int off = run;
        for (int w = 0; w < wv; ++w) off += s_wc[w];
        if (flag) {
            const int e = off + __popcll(m & ((1ull << lane) - 1));
            blist[2 * int64_t(e)] = r[6] + lx + ex * (ly + ey * lz);
            blist[2 * int64_t(e) + 1] = k;
        }
        run += s_wc[0] + s_wc[1] + s_wc[2] + s_wc[3];
        __syncthreads();
    }
}

// Axis cover rows (Img::axrow): one thread per coordinate of each axis, from the closed-form covers.
__global__ __launch_bounds__(256) void k_axis_rows(Geom g, int2 *__restrict__ axrow) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i >= g.W + g.H + g.D) return;
    const int a = i < g.W ? 0 : (i < g.W + g.H ? 1 : 2);
    const int x = a == 0 ? i : (a == 1 ? i - g.W : i - g.W - g.H);
    AxCov c[3];
    axis_cov<1>(g.ax[a], x, c);
    int codes = 0;
    for (int t = 0; t < 3; ++t) {
        const int d = c[t].cnt ? c[t].thi - c[1].thi + 1 : 1;   // in 0..2 on the axis (stride >= 1)
        codes |= (c[t].cnt | (d << 2)) << (4 * t);
    }
    axrow[i] = make_int2(c[1].thi, codes);
}

hipError_t launch_axis_rows(const Geom &g, int2 *axrow, hipStream_t s) {
    hipLaunchKernelGGL(k_axis_rows, dim3(blocks_for(int64_t(g.W) + g.H + g.D, 256)), dim3(256), 0, s, g, axrow);
    return hipGetLastError();
}

hipError_t launch_build_blist(const Geom &g, const int32_t *btab, int2 *blist, hipStream_t s) {
    hipLaunchKernelGGL(k_build_blist, dim3(unsigned(g.K)), dim3(256), 0, s, g, btab,
                       reinterpret_cast<int32_t *>(blist));
    return hipGetLastError();
}

hipError_t launch_setup_batch(int32_t conn, const Img *imgs, const SetupArg *args, const Item *rows, int32_t n_rows,
                              hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    return by_conn(conn, [&](auto c) { return conn_setup_batch<decltype(c)::value>(imgs, args, rows, n_rows, s); });
}

hipError_t launch_labels_batch(const Img *imgs, uint8_t *const *labels, const Item *rows, int32_t n_rows,
                               hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_labels_batch, dim3(unsigned(n_rows)), dim3(256), 0, s, imgs, labels, rows);
    return hipGetLastError();
}

hipError_t launch_validate(Ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

hipError_t launch_ctl_setup(Ctl *ctl, int32_t t_limit, int32_t stop_on_converge, int32_t clear_energy,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_setup, dim3(1), dim3(64), 0, s, ctl, t_limit, stop_on_converge, clear_energy);
    return hipGetLastError();
}

hipError_t launch_solve_phase(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return by_conn(grp.conn, [&](auto c) { return conn_solve<decltype(c)::value>(grp, s, e0, e1); });
}

hipError_t launch_consensus_phase(const Group &grp, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (grp.n_chk_items <= 0) return hipSuccess;
    return by_conn(grp.conn, [&](auto c) { return conn_consensus<decltype(c)::value>(grp, s, e0, e1); });
}

hipError_t launch_finalize_phase(const Group &grp, hipStream_t s, Ctl *mirror, int64_t seq) {
    const Img one = grp.one ? *grp.one : Img{};
    hipLaunchKernelGGL(k_finalize, dim3(unsigned(grp.n_imgs)), dim3(256), 0, s, grp.imgs, grp.queue, one,
                       int32_t(grp.one ? 1 : 0), grp.one ? mirror : nullptr, seq);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const Img *imgs, int32_t n, const int32_t *params, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_setup, dim3(blocks_for(n, 256)), dim3(256), 0, s, imgs, n, params);
    return hipGetLastError();
}

hipError_t launch_iteration(const Group &grp, hipStream_t s, Ctl *mirror, int64_t seq) {
    hipError_t e = launch_solve_phase(grp, s);
    if (e == hipSuccess) e = launch_consensus_phase(grp, s);
    if (e == hipSuccess) e = launch_finalize_phase(grp, s, mirror, seq);
    return e;
}

hipError_t launch_labels(const Geom &g, const int32_t *Y, uint8_t *labels, hipStream_t s) {
    const dim3 grid(blocks_for(g.W, 256), row_blocks(g));
    hipLaunchKernelGGL(k_labels, grid, dim3(256), 0, s, g, Y, labels);
    return hipGetLastError();
}

hipError_t launch_energy(const Geom &g, const int32_t *u, const int32_t *cw, const int32_t *Y, int64_t *part,
                         Ctl *ctl, hipStream_t s) {
    const int64_t rows = int64_t(g.H) * g.D;
    const unsigned wgs = unsigned(rows < ENERGY_WGS ? rows : ENERGY_WGS);
    const hipError_t e =
        by_conn(g.conn, [&](auto c) { return conn_energy<decltype(c)::value>(g, u, cw, Y, part, wgs, s); });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(256), 0, s, part, int(wgs), ctl);
    return hipGetLastError();
}

#endif  // DOPE_CONN

}  // namespace dope
