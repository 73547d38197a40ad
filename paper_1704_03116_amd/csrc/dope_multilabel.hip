// Multi-label Potts segmentation by alpha-expansion around DOPE (include/dope.h, dope_ml_*).
//
// Energy: E(L) = sum_i D[L_i, i] + sum_{edges (i,j)} V_ij [L_i != L_j] (integers, lambda folded into V).  The
// expansion move of label a lets every pixel keep its label or switch to a; with l_i(0) = L_i, l_i(1) = a, twice
// the move's energy is 2 E(L) + sum_i u_i y_i + sum_edges W_ij |y_i - y_j| where
//   u_i  = 2 (D[a, i] - D[L_i, i]) - sum_{j ~ i : L_j != L_i, L_i != a} V_ij (1 + [L_j = a]),
//   W_ij = 2 V_ij if L_i = L_j != a;  V_ij if L_i != L_j and neither is a;  0 otherwise
// (each edge term [l_i(y_i) != l_j(y_j)], doubled, is affine in y plus a multiple of |y_i - y_j|).  That is the
// binary energy of Eq. (1) with lambda = 1 and w = W >= 0, which a DOPE context solves (Algorithm 1 to its
// stopping rule); the move's labelling is kept only when it lowers E.
//
// Kernels: the move's binary energy (one thread per pixel, all full-stencil neighbours), the move's labelling
// together with its energy (one pass: a neighbour's new label is y_j ? a : L_j), the initial labels (argmin of D).
// Everything is integer; E is an int64 sum of per-workgroup partials added with one atomic per workgroup.
#include "../../include/dope.h"

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace {

constexpr int ML_NT = 256;
constexpr int ML_MAX_HALF = 64;

struct MlGeom {
    int32_t W, H, D;
    int32_t h;
    int32_t nl;
    int64_t n;
    int4 off[ML_MAX_HALF];   // half-stencil offsets (dx, dy, dz, linear)
};

__device__ __forceinline__ bool ml_in(const MlGeom &g, int x, int y, int z) {
    return x >= 0 && x < g.W && y >= 0 && y < g.H && z >= 0 && z < g.D;
}

// L_i = argmin_l D[l, i] (smallest l on ties)
__global__ __launch_bounds__(ML_NT) void k_ml_init(const MlGeom g, const int32_t *__restrict__ Dt,
                                                   uint8_t *__restrict__ L) {
    const int64_t i = int64_t(blockIdx.x) * ML_NT + threadIdx.x;
    if (i >= g.n) return;
    int32_t best = Dt[i];
    int lab = 0;
    for (int l = 1; l < g.nl; ++l) {
        const int32_t v = Dt[int64_t(l) * g.n + i];
        if (v < best) { best = v; lab = l; }
    }
    L[i] = uint8_t(lab);
}

// Validation: bit 0 = a negative weight, bit 1 = a nonzero weight on an off-grid edge, bit 2 = a data term of
// magnitude 2^26 or more or a weight above 2^20 (then every move unary, |2 dD| + 2 sum_j V_ij over at most 122
// neighbours, fits int32).
constexpr int32_t ML_D_LIMIT = 1 << 26;
constexpr int32_t ML_V_LIMIT = 1 << 20;
__global__ __launch_bounds__(ML_NT) void k_ml_validate(const MlGeom g, const int32_t *__restrict__ Dt,
                                                       const int32_t *__restrict__ V, int32_t *__restrict__ flags) {
    const int64_t i = int64_t(blockIdx.x) * ML_NT + threadIdx.x;
    if (i >= g.n) return;
    const int x = int(i % g.W), y = int((i / g.W) % g.H), z = int(i / (int64_t(g.W) * g.H));
    int f = 0;
    for (int o = 0; o < g.h; ++o) {
        const int32_t v = V[int64_t(o) * g.n + i];
        if (v < 0) f |= 1;
        if (v > ML_V_LIMIT) f |= 4;
        if (v != 0 && !ml_in(g, x + g.off[o].x, y + g.off[o].y, z + g.off[o].z)) f |= 2;
    }
    for (int l = 0; l < g.nl; ++l) {
        const int32_t d = Dt[int64_t(l) * g.n + i];
        if (d >= ML_D_LIMIT || d <= -ML_D_LIMIT) f |= 4;
    }
    if (f) atomicOr(flags, f);
}

// Binary energy of the expansion move of label a (see the file header): u[i], and w[o][i] for the edge
// i <-> i + off[o].
__global__ __launch_bounds__(ML_NT) void k_ml_move(const MlGeom g, const int32_t *__restrict__ Dt,
                                                   const int32_t *__restrict__ V, const uint8_t *__restrict__ L,
                                                   int32_t a, int32_t *__restrict__ u, int32_t *__restrict__ w) {
    const int64_t i = int64_t(blockIdx.x) * ML_NT + threadIdx.x;
    if (i >= g.n) return;
    const int x = int(i % g.W), y = int((i / g.W) % g.H), z = int(i / (int64_t(g.W) * g.H));
    const int li = L[i];
    int64_t ui = 2 * (int64_t(Dt[int64_t(a) * g.n + i]) - int64_t(Dt[int64_t(li) * g.n + i]));
    for (int o = 0; o < g.h; ++o) {
        const int4 v = g.off[o];
        // forward neighbour i + off: the half-edge this pixel owns
        int32_t wf = 0;
        if (ml_in(g, x + v.x, y + v.y, z + v.z)) {
            const int64_t j = i + v.w;
            const int lj = L[j];
            const int32_t c = V[int64_t(o) * g.n + i];
            if (li == lj) wf = li != a ? 2 * c : 0;
            else wf = (li != a && lj != a) ? c : 0;
            if (li != lj && li != a) ui -= int64_t(c) * (lj == a ? 2 : 1);
        }
        w[int64_t(o) * g.n + i] = wf;
        // backward neighbour i - off: only the unary share of pixel i
        if (ml_in(g, x - v.x, y - v.y, z - v.z)) {
            const int64_t j = i - v.w;
            const int lj = L[j];
            const int32_t c = V[int64_t(o) * g.n + j];
            if (li != lj && li != a) ui -= int64_t(c) * (lj == a ? 2 : 1);
        }
    }
    // |u_i| <= 2 |dD| + 2 sum_j V_ij < 2^31 under the limits k_ml_validate enforces
    u[i] = int32_t(ui);
}

// Labels after the move (a >= 0: L'_i = y_i ? a : L_i; a < 0: L unchanged) and their energy E(L'), accumulated
// into *acc (zeroed beforehand).
__global__ __launch_bounds__(ML_NT) void k_ml_apply(const MlGeom g, const int32_t *__restrict__ Dt,
                                                    const int32_t *__restrict__ V, const uint8_t *__restrict__ L,
                                                    const uint8_t *__restrict__ yb, int32_t a,
                                                    uint8_t *__restrict__ Lout, unsigned long long *acc) {
    __shared__ long long part[ML_NT / 64];
    const int64_t i = int64_t(blockIdx.x) * ML_NT + threadIdx.x;
    long long e = 0;
    if (i < g.n) {
        const int x = int(i % g.W), y = int((i / g.W) % g.H), z = int(i / (int64_t(g.W) * g.H));
        const int li = (a >= 0 && yb[i]) ? a : L[i];
        Lout[i] = uint8_t(li);
        e = Dt[int64_t(li) * g.n + i];
        for (int o = 0; o < g.h; ++o) {
            const int4 v = g.off[o];
            if (!ml_in(g, x + v.x, y + v.y, z + v.z)) continue;
            const int64_t j = i + v.w;
            const int lj = (a >= 0 && yb[j]) ? a : L[j];
            if (li != lj) e += V[int64_t(o) * g.n + i];
        }
    }
    for (int s = 32; s >= 1; s >>= 1) e += __shfl_xor(e, s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int k = 0; k < ML_NT / 64; ++k) t += part[k];
        atomicAdd(acc, (unsigned long long)t);
    }
}

__global__ void k_ml_zero(unsigned long long *acc, int32_t *flags) {
    *acc = 0;
    *flags = 0;
}

std::vector<int4> half_offsets(int ndim, int conn, int W, int H) {
    std::vector<int4> out;
    auto add = [&](int dx, int dy, int dz) { out.push_back(make_int4(dx, dy, dz, dx + W * (dy + H * dz))); };
    if (ndim == 2 && conn == 4) { add(1, 0, 0); add(0, 1, 0); }
    else if (ndim == 2 && conn == 8) { add(1, 0, 0); add(0, 1, 0); add(1, 1, 0); add(-1, 1, 0); }
    else if (ndim == 2 && (conn == 24 || conn == 48 || conn == 80)) {
        const int r = conn == 24 ? 2 : (conn == 48 ? 3 : 4);
        for (int dx = 1; dx <= r; ++dx) add(dx, 0, 0);
        for (int dy = 1; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) add(dx, dy, 0);
    } else if (ndim == 3 && conn == 6) { add(1, 0, 0); add(0, 1, 0); add(0, 0, 1); }
    else if (ndim == 3 && (conn == 32 || conn == 122)) {
        const int r = conn == 32 ? 2 : 3;
        for (int dz = 0; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    const int d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 == 0 || d2 > r * r) continue;
                    if (dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0)))) add(dx, dy, dz);
                }
    }
    return out;
}

}  // namespace

struct dope_ml {
    dope_params p{};
    MlGeom g{};
    dope_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t *Dt = nullptr, *V = nullptr, *u = nullptr, *w = nullptr, *flags = nullptr;
    uint8_t *L = nullptr, *Ln = nullptr, *y = nullptr;
    unsigned long long *acc = nullptr;
    int64_t energy = 0;
    bool energy_set = false;
    dope_ml_info info{};
    std::string err;
};

namespace {

dope_status mlfail(dope_ml *m, dope_status s, const std::string &msg) {
    if (m) m->err = msg;
    return s;
}

#define ML_HIP(m, expr, what)                                                                  \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return mlfail(m, DOPE_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e));  \
        }                                                                                      \
    } while (0)

unsigned ml_blocks(int64_t n) { return unsigned((n + ML_NT - 1) / ML_NT); }

// Labels after the move of label a into Ln (a < 0: a copy of L) and their energy E, read back to *out.
dope_status ml_energy_of(dope_ml *m, int32_t a, int64_t *out) {
    hipLaunchKernelGGL(k_ml_zero, dim3(1), dim3(1), 0, m->stream, m->acc, m->flags);
    hipLaunchKernelGGL(k_ml_apply, dim3(ml_blocks(m->g.n)), dim3(ML_NT), 0, m->stream, m->g, m->Dt, m->V, m->L,
                       m->y, a, m->Ln, m->acc);
    ML_HIP(m, hipGetLastError(), "energy launch");
    unsigned long long h = 0;
    ML_HIP(m, hipMemcpyAsync(&h, m->acc, sizeof(h), hipMemcpyDeviceToHost, m->stream), "energy readback");
    ML_HIP(m, hipStreamSynchronize(m->stream), "stream synchronize");
    *out = int64_t(h);
    return DOPE_OK;
}

}  // namespace

extern "C" {

dope_status dope_ml_create(const dope_params *p, int32_t n_labels, dope_ml **out) {
    if (!p || !out) return DOPE_EINVAL;
    *out = nullptr;
    if (n_labels < 2 || n_labels > 255) return DOPE_EINVAL;
    dope_params q = *p;
    q.solver = DOPE_SOLVER_MAXFLOW;   // every move is submodular
    // the expansion kernels and the binary solves share one stream (the caller's, or one of our own)
    bool own_stream = false;
    if (!q.stream) {
        hipStream_t s = nullptr;
        if (hipStreamCreate(&s) != hipSuccess) {
            (void)hipGetLastError();
            return DOPE_EDEVICE;
        }
        q.stream = s;
        own_stream = true;
    }
    dope_ctx *ctx = nullptr;
    dope_status st = dope_create(&q, &ctx);
    dope_ml *m = st == DOPE_OK ? new (std::nothrow) dope_ml() : nullptr;
    if (!m) {
        if (ctx) dope_destroy(ctx);
        if (own_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(q.stream));
        return st == DOPE_OK ? DOPE_ENOMEM : st;
    }
    m->p = q;
    m->ctx = ctx;
    m->stream = static_cast<hipStream_t>(q.stream);
    m->own_stream = own_stream;
    int64_t n = 0;
    int32_t K = 0, h = 0;
    int64_t tot = 0;
    dope_sizes(ctx, &n, &K, &tot, &h);
    const std::vector<int4> offs = half_offsets(q.ndim, q.connectivity, q.dims[0], q.dims[1]);
    if (int(offs.size()) != h || h > ML_MAX_HALF) {
        dope_ml_destroy(m);
        return DOPE_EINVAL;
    }
    m->g.W = q.dims[0];
    m->g.H = q.dims[1];
    m->g.D = q.ndim == 3 ? q.dims[2] : 1;
    m->g.h = h;
    m->g.nl = n_labels;
    m->g.n = n;
    for (int o = 0; o < h; ++o) m->g.off[o] = offs[size_t(o)];
    const size_t bytes_D = size_t(n_labels) * size_t(n) * 4, bytes_V = size_t(h) * size_t(n) * 4;
    void *ptr = nullptr;
    if (hipMalloc(&ptr, bytes_D + 2 * bytes_V + size_t(n) * 4 + 3 * size_t(n) + 512) != hipSuccess) {
        (void)hipGetLastError();
        dope_ml_destroy(m);
        return DOPE_ENOMEM;
    }
    char *b = static_cast<char *>(ptr);
    m->acc = reinterpret_cast<unsigned long long *>(b);
    m->flags = reinterpret_cast<int32_t *>(b + 256);
    b += 512;
    m->Dt = reinterpret_cast<int32_t *>(b);
    b += bytes_D;
    m->V = reinterpret_cast<int32_t *>(b);
    b += bytes_V;
    m->w = reinterpret_cast<int32_t *>(b);
    b += bytes_V;
    m->u = reinterpret_cast<int32_t *>(b);
    b += size_t(n) * 4;
    m->L = reinterpret_cast<uint8_t *>(b);
    m->Ln = m->L + n;
    m->y = m->Ln + n;
    *out = m;
    return DOPE_OK;
}

dope_status dope_ml_set_energy(dope_ml *m, const int32_t *D, const int32_t *V, int32_t mem_kind) {
    if (!m || !D || !V) return DOPE_EINVAL;
    if (mem_kind != DOPE_MEM_HOST && mem_kind != DOPE_MEM_DEVICE) return mlfail(m, DOPE_EINVAL, "bad mem_kind");
    m->energy_set = false;
    const hipMemcpyKind kind = mem_kind == DOPE_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const int64_t n = m->g.n;
    ML_HIP(m, hipMemcpyAsync(m->Dt, D, size_t(m->g.nl) * size_t(n) * 4, kind, m->stream), "D upload");
    ML_HIP(m, hipMemcpyAsync(m->V, V, size_t(m->g.h) * size_t(n) * 4, kind, m->stream), "V upload");
    hipLaunchKernelGGL(k_ml_zero, dim3(1), dim3(1), 0, m->stream, m->acc, m->flags);
    hipLaunchKernelGGL(k_ml_validate, dim3(ml_blocks(n)), dim3(ML_NT), 0, m->stream, m->g, m->Dt, m->V, m->flags);
    hipLaunchKernelGGL(k_ml_init, dim3(ml_blocks(n)), dim3(ML_NT), 0, m->stream, m->g, m->Dt, m->L);
    ML_HIP(m, hipGetLastError(), "set-up launch");
    int32_t flags = 0;
    ML_HIP(m, hipMemcpyAsync(&flags, m->flags, 4, hipMemcpyDeviceToHost, m->stream), "validation readback");
    ML_HIP(m, hipStreamSynchronize(m->stream), "stream synchronize");
    if (flags & 1) return mlfail(m, DOPE_ENOTSUBMODULAR, "negative Potts weight");
    if (flags & 2) return mlfail(m, DOPE_EINVAL, "nonzero weight on an off-grid edge");
    if (flags & 4) return mlfail(m, DOPE_EINVAL, "data term |D| >= 2^26 or Potts weight > 2^20");
    int64_t e = 0;
    dope_status st = ml_energy_of(m, -1, &e);
    if (st != DOPE_OK) return st;
    m->energy = e;
    m->info = dope_ml_info{};
    m->info.energy = e;
    m->energy_set = true;
    m->err.clear();
    return DOPE_OK;
}

dope_status dope_ml_step(dope_ml *m, int32_t label, int32_t *accepted, int64_t *energy) {
    if (!m) return DOPE_EINVAL;
    if (!m->energy_set) return mlfail(m, DOPE_ESTATE, "dope_ml_set_energy has not been called");
    if (label < 0 || label >= m->g.nl) return mlfail(m, DOPE_EINVAL, "label out of range");
    const int64_t n = m->g.n;
    hipLaunchKernelGGL(k_ml_move, dim3(ml_blocks(n)), dim3(ML_NT), 0, m->stream, m->g, m->Dt, m->V, m->L, label,
                       m->u, m->w);
    ML_HIP(m, hipGetLastError(), "move launch");
    dope_status st = dope_set_energy_async(m->ctx, m->u, m->w, 256, DOPE_MEM_DEVICE);
    dope_info bi{};
    if (st == DOPE_OK) st = dope_solve(m->ctx, &bi);
    if (st == DOPE_OK) st = dope_labels(m->ctx, m->y, DOPE_MEM_DEVICE);
    if (st != DOPE_OK) return mlfail(m, st, std::string("binary move: ") + dope_last_error(m->ctx));
    int64_t e = 0;
    st = ml_energy_of(m, label, &e);
    if (st != DOPE_OK) return st;
    const bool acc = e < m->energy;
    if (acc) {
        uint8_t *t = m->L;
        m->L = m->Ln;
        m->Ln = t;
        m->energy = e;
        ++m->info.accepted;
    }
    ++m->info.moves;
    m->info.binary_iterations += bi.iters_done;
    m->info.energy = m->energy;
    if (accepted) *accepted = acc ? 1 : 0;
    if (energy) *energy = m->energy;
    return DOPE_OK;
}

dope_status dope_ml_solve(dope_ml *m, int32_t max_cycles, dope_ml_info *out) {
    if (!m) return DOPE_EINVAL;
    if (!m->energy_set) return mlfail(m, DOPE_ESTATE, "dope_ml_set_energy has not been called");
    if (max_cycles < 0) return mlfail(m, DOPE_EINVAL, "max_cycles must be >= 0");
    for (int c = 0; c < max_cycles; ++c) {
        bool changed = false;
        for (int a = 0; a < m->g.nl; ++a) {
            int32_t acc = 0;
            dope_status st = dope_ml_step(m, a, &acc, nullptr);
            if (st != DOPE_OK) return st;
            changed = changed || acc;
        }
        ++m->info.cycles;
        if (!changed) break;
    }
    if (out) *out = m->info;
    return DOPE_OK;
}

dope_status dope_ml_labels(dope_ml *m, uint8_t *labels, int32_t mem_kind) {
    if (!m || !labels) return DOPE_EINVAL;
    if (!m->energy_set) return mlfail(m, DOPE_ESTATE, "dope_ml_set_energy has not been called");
    if (mem_kind == DOPE_MEM_DEVICE) {
        ML_HIP(m, hipMemcpyAsync(labels, m->L, size_t(m->g.n), hipMemcpyDeviceToDevice, m->stream), "labels copy");
        return DOPE_OK;
    }
    ML_HIP(m, hipMemcpyAsync(labels, m->L, size_t(m->g.n), hipMemcpyDeviceToHost, m->stream), "labels copy");
    ML_HIP(m, hipStreamSynchronize(m->stream), "stream synchronize");
    return DOPE_OK;
}

dope_status dope_ml_info_get(dope_ml *m, dope_ml_info *out) {
    if (!m || !out) return DOPE_EINVAL;
    *out = m->info;
    return DOPE_OK;
}

const char *dope_ml_last_error(const dope_ml *m) { return m ? m->err.c_str() : ""; }

void dope_ml_destroy(dope_ml *m) {
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    if (m->acc) (void)hipFree(m->acc);
    if (m->ctx) dope_destroy(m->ctx);
    if (m->own_stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

}  // extern "C"
