"""Thin Python wrapper over the C ABI: owns a dope_ctx and marshals numpy arrays (host) or torch tensors
(device) into the library's entry points.  No arithmetic of the method happens here."""
import ctypes

import numpy as np

from . import _native as N


def _ptr(a):
    """Data pointer and memory kind of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return ctypes.c_void_p(a.ctypes.data), N.DOPE_MEM_HOST
    import torch
    if not isinstance(a, torch.Tensor) or not a.is_contiguous():
        raise ValueError("expected a contiguous numpy array or torch tensor")
    return ctypes.c_void_p(a.data_ptr()), (N.DOPE_MEM_DEVICE if a.is_cuda else N.DOPE_MEM_HOST)


def make_params(dims, connectivity, block, overlap, mu0, *, ndim=None, mu_fact=(21, 20), eps_q16=6554,
                max_iter=50, solver="auto"):
    p = N.dope_params()
    dims = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
    p.ndim = ndim if ndim is not None else (3 if connectivity in (6, 32, 122, 256) else 2)
    p.dims[:] = dims
    p.connectivity = int(connectivity)
    p.block[:] = tuple(int(b) for b in block) + (1,) * (3 - len(block))
    p.overlap[:] = tuple(int(o) for o in overlap) + (0,) * (3 - len(overlap))
    p.mu0 = int(mu0)
    p.mu_fact_num, p.mu_fact_den = int(mu_fact[0]), int(mu_fact[1])
    p.eps_q16 = int(eps_q16)
    p.max_iter = int(max_iter)
    p.solver = {"auto": N.DOPE_SOLVER_AUTO, "maxflow": N.DOPE_SOLVER_MAXFLOW,
                "exhaustive": N.DOPE_SOLVER_EXHAUSTIVE, "lsatr": N.DOPE_SOLVER_LSATR}[solver]
    return p


def params_from_problem(prob, block=None, overlap=None):
    return make_params(prob.dims, prob.conn, block if block is not None else prob.block,
                       overlap if overlap is not None else prob.overlap, prob.mu0, ndim=prob.ndim,
                       mu_fact=(prob.mu_num, prob.mu_den), eps_q16=prob.eps_q16, max_iter=prob.max_iter,
                       solver=prob.solver)


def autotune(ndim, dims, connectivity):
    """(block, overlap) chosen by the library for this image shape (pure function of shape and stencil)."""
    d = (ctypes.c_int32 * 3)(*(tuple(int(x) for x in dims) + (1,) * (3 - len(dims))))
    b = (ctypes.c_int32 * 3)()
    o = (ctypes.c_int32 * 3)()
    N.check(N.dope_autotune(int(ndim), d, int(connectivity), b, o))
    return tuple(b), tuple(o)


def dispatch_order(params):
    """dope_dispatch_order: the block each workgroup of a one-image block-solve launch takes (int32 numpy array)."""
    K = ctypes.c_int32()
    N.check(N.dope_dispatch_order(ctypes.byref(params), ctypes.byref(K), None))
    order = np.zeros(K.value, dtype=np.int32)
    N.check(N.dope_dispatch_order(ctypes.byref(params), ctypes.byref(K), ctypes.c_void_p(order.ctypes.data)))
    return order


def solve_noalloc(params, u, w, lambda_q8, labels, stream=None):
    """dope_solve_noalloc: one whole solve whose device state lives in the library's static device array.
    u, w, labels are device tensors; returns the loop information (dict).  stream: HIP stream handle (None = the
    current torch stream)."""
    p = N.dope_params()
    ctypes.memmove(ctypes.byref(p), ctypes.byref(params), ctypes.sizeof(p))
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    p.stream = ctypes.c_void_p(stream) if stream else None
    up, uk = _ptr(u)
    wp, wk = _ptr(w)
    lp, lk = _ptr(labels)
    if not (uk == wk == lk == N.DOPE_MEM_DEVICE):
        raise ValueError("dope_solve_noalloc takes device tensors")
    info = N.dope_info()
    st = N.dope_solve_noalloc(ctypes.byref(p), up, wp, int(lambda_q8), lp, ctypes.byref(info))
    if st != N.DOPE_OK:
        raise N.DopeError(st, N.dope_last_error(None).decode())
    return _info(info)


def measure_lds_bandwidth(reps=2000, stream=None):
    """dope_measure_lds_bandwidth: measured LDS read bandwidth of the GPU, with the nominal 128 bytes per clock
    and CU (256 CUs at 2.4 GHz) beside it."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    out = ctypes.c_double()
    N.check(N.dope_measure_lds_bandwidth(ctypes.c_void_p(stream) if stream else None, int(reps), ctypes.byref(out)))
    return {"gbs": round(out.value / 1e9, 1), "reps": int(reps),
            "nominal_gbs_128B_per_clk_per_cu": round(128 * 256 * 2.4e9 / 1e9, 1)}


class Dope:
    """One DOPE solve context (see include/dope.h)."""

    def __init__(self, dims, connectivity, block, overlap, mu0, *, ndim=None, mu_fact=(21, 20), eps_q16=6554,
                 max_iter=50, solver="auto", stream=None, torch_workspace=True):
        p = make_params(dims, connectivity, block, overlap, mu0, ndim=ndim, mu_fact=mu_fact, eps_q16=eps_q16,
                        max_iter=max_iter, solver=solver)
        self._workspace = None
        if stream is None and torch_workspace:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        p.stream = ctypes.c_void_p(stream) if stream else None
        self.params = p
        ctx = ctypes.c_void_p()
        st = N.dope_create(ctypes.byref(p), ctypes.byref(ctx))
        if st != N.DOPE_OK:
            raise N.DopeError(st, N.dope_last_error(None).decode())
        self.ctx = ctx
        n = ctypes.c_int64()
        K = ctypes.c_int32()
        tot = ctypes.c_int64()
        h = ctypes.c_int32()
        N.check(N.dope_sizes(ctx, ctypes.byref(n), ctypes.byref(K), ctypes.byref(tot), ctypes.byref(h)), ctx)
        self.n, self.K, self.tot, self.h = n.value, K.value, tot.value, h.value
        if torch_workspace:
            import torch
            nbytes = N.dope_workspace_bytes(ctypes.byref(p))
            # torch's caching allocator returns 256-byte aligned blocks
            self._workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._workspace.data_ptr()
            aligned = (base + 255) & ~255
            N.check(N.dope_bind_workspace(ctx, ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes)), ctx)

    @classmethod
    def from_problem(cls, prob, **kw):
        kw.setdefault("mu_fact", (prob.mu_num, prob.mu_den))
        kw.setdefault("eps_q16", prob.eps_q16)
        kw.setdefault("max_iter", prob.max_iter)
        kw.setdefault("solver", prob.solver)
        return cls(prob.dims, prob.conn, prob.block, prob.overlap, prob.mu0, ndim=prob.ndim, **kw)

    def close(self):
        if self.ctx:
            N.dope_destroy(self.ctx)
            self.ctx = None
            self._workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- entry points ----
    def set_energy(self, u, w, lambda_q8):
        pu, ku = _ptr(u)
        pw, kw = _ptr(w)
        if ku != kw:
            raise ValueError("u and w must live in the same memory")
        N.check(N.dope_set_energy(self.ctx, pu, pw, int(lambda_q8), ku), self.ctx)

    def set_energy_async(self, u, w, lambda_q8):
        pu, ku = _ptr(u)
        pw, kw = _ptr(w)
        if ku != kw:
            raise ValueError("u and w must live in the same memory")
        N.check(N.dope_set_energy_async(self.ctx, pu, pw, int(lambda_q8), ku), self.ctx)

    def iterate(self, n_iter=1):
        info = N.dope_info()
        N.check(N.dope_iterate(self.ctx, int(n_iter), ctypes.byref(info)), self.ctx)
        return _info(info)

    def iterate_status(self, n_iter=1):
        """Like iterate() but returns (status, info) instead of raising."""
        info = N.dope_info()
        st = N.dope_iterate(self.ctx, int(n_iter), ctypes.byref(info))
        return st, _info(info)

    def solve(self):
        info = N.dope_info()
        N.check(N.dope_solve(self.ctx, ctypes.byref(info)), self.ctx)
        return _info(info)

    def iterate_metrics(self, n_iter, path=None):
        """Runs up to n_iter iterations one at a time and returns one record per iteration: t, status, the
        stopping test (max_k r_k, converged), mu, and the block solves' statistics (free nodes after the strict
        forcing test, push-relabel rounds, global relabels, elimination passes: sum and max over blocks) with the
        block of the largest residual.  Stops after the iteration that meets the stopping test (Algorithm 1's while-condition), when
        the loop halts (t no longer advances) or when an iteration fails.  path: also written there as JSON
        lines."""
        import json
        out = []
        fh = open(path, "w") if path else None
        try:
            t_prev = None
            for _ in range(int(n_iter)):
                status, info = self.iterate_status(1)
                if status != N.DOPE_OK:
                    out.append({"t": info["iters_done"], "status": int(status)})
                    if fh:
                        fh.write(json.dumps(out[-1]) + "\n")
                    break
                if info["iters_done"] == t_prev:
                    break
                t_prev = info["iters_done"]
                st = self.block_stats()
                r = self.block_resid()
                rec = {"t": info["iters_done"], "status": 0, "max_resid2": int(info["max_resid2"]),
                       "converged": info["converged"], "mu": int(info["mu"]),
                       "worst_block": int(np.argmax(r)) if len(r) else -1,
                       "free_nodes": {"sum": int(st[:, 0].sum()), "max": int(st[:, 0].max())},
                       "pushrelabel_rounds": {"sum": int(st[:, 1].sum()), "max": int(st[:, 1].max())},
                       "global_relabels_max": int(st[:, 2].max()),
                       "elimination_passes_max": int(st[:, 3].max())}
                out.append(rec)
                if fh:
                    fh.write(json.dumps(rec) + "\n")
                if rec["converged"]:
                    break
        finally:
            if fh:
                fh.close()
        return out

    def labels(self, out=None):
        if out is None:
            out = np.zeros(self.n, dtype=np.uint8)
        p, k = _ptr(out)
        N.check(N.dope_labels(self.ctx, p, k), self.ctx)
        return out

    def energy(self):
        e = ctypes.c_int64()
        N.check(N.dope_energy(self.ctx, ctypes.byref(e)), self.ctx)
        return e.value

    def get_state(self):
        Y = np.zeros(self.n, dtype=np.int32)
        A = np.zeros(self.tot, dtype=np.int32)
        yh = np.zeros(self.tot, dtype=np.uint8)
        mu = ctypes.c_int64()
        t = ctypes.c_int32()
        N.check(N.dope_get_state(self.ctx, ctypes.c_void_p(Y.ctypes.data), ctypes.c_void_p(A.ctypes.data),
                                 ctypes.c_void_p(yh.ctypes.data), ctypes.byref(mu), ctypes.byref(t)), self.ctx)
        return Y, A, yh, mu.value, t.value

    def set_state(self, Y, A, yhat, mu, t):
        Y = np.ascontiguousarray(Y, dtype=np.int32)
        A = np.ascontiguousarray(A, dtype=np.int32)
        yhat = np.ascontiguousarray(yhat, dtype=np.uint8)
        N.check(N.dope_set_state(self.ctx, ctypes.c_void_p(Y.ctypes.data), ctypes.c_void_p(A.ctypes.data),
                                 ctypes.c_void_p(yhat.ctypes.data), int(mu), int(t)), self.ctx)

    def block_resid(self):
        r = np.zeros(self.K, dtype=np.int64)
        N.check(N.dope_block_resid(self.ctx, ctypes.c_void_p(r.ctypes.data)), self.ctx)
        return r

    def block_stats(self):
        s = np.zeros((self.K, 4), dtype=np.int32)
        N.check(N.dope_block_stats(self.ctx, ctypes.c_void_p(s.ctypes.data)), self.ctx)
        return s

    def block_table(self):
        K = ctypes.c_int32()
        tab = np.zeros((self.K, 7), dtype=np.int32)
        N.check(N.dope_block_table(self.ctx, ctypes.byref(K), ctypes.c_void_p(tab.ctypes.data)), self.ctx)
        return tab

    def profile_enable(self, on=True):
        N.check(N.dope_profile_enable(self.ctx, 1 if on else 0), self.ctx)

    def profile_read(self):
        sm, cm = ctypes.c_double(), ctypes.c_double()
        sl, cl = ctypes.c_int32(), ctypes.c_int32()
        N.check(N.dope_profile_read(self.ctx, ctypes.byref(sm), ctypes.byref(sl), ctypes.byref(cm),
                                    ctypes.byref(cl)), self.ctx)
        return {"solve_ms": sm.value, "solve_launches": sl.value, "consensus_ms": cm.value,
                "consensus_launches": cl.value}


def _info(info):
    return {"iters_done": info.iters_done, "converged": bool(info.converged), "max_resid2": info.max_resid2,
            "mu": info.mu}


class Batch:
    """A dope_batch over existing Dope contexts (which must outlive it)."""

    def __init__(self, members, graph=False, workers=0):
        self.members = list(members)
        arr = (ctypes.c_void_p * len(self.members))(*[m.ctx.value for m in self.members])
        b = ctypes.c_void_p()
        st = N.dope_batch_create(arr, len(self.members), ctypes.byref(b))
        if st != N.DOPE_OK:
            raise N.DopeError(st, N.dope_last_error(self.members[0].ctx).decode())
        self.b = b
        if graph:
            self._check(N.dope_batch_set_graph(b, 1))
        if workers:
            self._check(N.dope_batch_set_workers(b, int(workers)))

    def _check(self, st):
        if st != N.DOPE_OK:
            raise N.DopeError(st, N.dope_batch_last_error(self.b).decode())

    def set_energy_async(self, us, ws, lambdas_q8):
        """Energy upload of every member in one launch (device tensors or host arrays, all in the same memory)."""
        n = len(self.members)
        if not (len(us) == len(ws) == len(lambdas_q8) == n):
            raise ValueError("one u, w and lambda per member")
        pu, pw, kinds = [], [], set()
        for u, w in zip(us, ws):
            a, ka = _ptr(u)
            c, kc = _ptr(w)
            pu.append(a)
            pw.append(c)
            kinds.update((ka, kc))
        if len(kinds) != 1:
            raise ValueError("all inputs must live in the same memory")
        self._keep = (us, ws)   # device inputs must stay alive until the upload has run
        arr_u = (ctypes.c_void_p * n)(*[x.value for x in pu])
        arr_w = (ctypes.c_void_p * n)(*[x.value for x in pw])
        lam = (ctypes.c_int32 * n)(*[int(x) for x in lambdas_q8])
        self._check(N.dope_batch_set_energy_async(self.b, arr_u, arr_w, lam, kinds.pop()))

    def labels(self, outs=None):
        """Labels of every member in one launch: into the given device tensors (stream-ordered), or returned as host
        arrays."""
        n = len(self.members)
        if outs is None:
            outs = [np.empty(m.n, dtype=np.uint8) for m in self.members]
            arr = (ctypes.c_void_p * n)(*[o.ctypes.data for o in outs])
            self._check(N.dope_batch_labels(self.b, arr, N.DOPE_MEM_HOST))
            return outs
        arr = (ctypes.c_void_p * n)(*[int(o.data_ptr()) for o in outs])
        self._check(N.dope_batch_labels(self.b, arr, N.DOPE_MEM_DEVICE))
        return outs

    def iterate(self, n_iter=1):
        self._check(N.dope_batch_iterate(self.b, int(n_iter)))

    def iterate_status(self, n_iter=1):
        return N.dope_batch_iterate(self.b, int(n_iter))

    def solve(self):
        self._check(N.dope_batch_solve(self.b))

    def info(self):
        arr = (N.dope_info * len(self.members))()
        self._check(N.dope_batch_info(self.b, arr))
        return [_info(x) for x in arr]

    def close(self):
        if getattr(self, "b", None):
            N.dope_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A dope_server: FIFO admission by HBM footprint, iters_per_step batched iterations per step()."""

    def __init__(self, hbm_budget, max_active, iters_per_step=1):
        sp = N.dope_server_params()
        sp.hbm_budget = int(hbm_budget)
        sp.max_active = int(max_active)
        sp.iters_per_step = int(iters_per_step)
        sp.stream = None
        s = ctypes.c_void_p()
        st = N.dope_server_create(ctypes.byref(sp), ctypes.byref(s))
        if st != N.DOPE_OK:
            raise N.DopeError(st, "dope_server_create failed")
        self.s = s
        self._held = {}   # ticket -> borrowed buffers kept alive until the request finishes

    def _check(self, st):
        if st != N.DOPE_OK:
            raise N.DopeError(st, N.dope_server_last_error(self.s).decode())

    def submit(self, params, u, w, lambda_q8, labels_out):
        pu, ku = _ptr(u)
        pw, kw = _ptr(w)
        pl, kl = _ptr(labels_out)
        t = ctypes.c_int64()
        self._check(N.dope_server_submit(self.s, ctypes.byref(params), pu, pw, int(lambda_q8), ku, pl, kl,
                                         ctypes.byref(t)))
        self._held[t.value] = (u, w, labels_out)
        return t.value

    def step(self, max_finished=4096):
        buf = (ctypes.c_int64 * max_finished)()
        nf = ctypes.c_int32()
        self._check(N.dope_server_step(self.s, buf, max_finished, ctypes.byref(nf)))
        done = [buf[i] for i in range(min(nf.value, max_finished))]
        for t in done:
            self._held.pop(t, None)
        return done

    def result(self, ticket):
        info = N.dope_info()
        st = ctypes.c_int32()
        self._check(N.dope_server_result(self.s, int(ticket), ctypes.byref(info), ctypes.byref(st)))
        return st.value, _info(info)

    def load(self):
        w, a = ctypes.c_int32(), ctypes.c_int32()
        used = ctypes.c_size_t()
        self._check(N.dope_server_load(self.s, ctypes.byref(w), ctypes.byref(a), ctypes.byref(used)))
        return w.value, a.value, used.value

    def close(self):
        if getattr(self, "s", None):
            N.dope_server_destroy(self.s)
            self.s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiLabel:
    """A dope_ml: multi-label Potts segmentation by alpha-expansion around DOPE (see include/dope.h)."""

    def __init__(self, dims, connectivity, block, overlap, mu0, n_labels, *, ndim=None, mu_fact=(21, 20),
                 eps_q16=6554, max_iter=50, stream=None):
        p = make_params(dims, connectivity, block, overlap, mu0, ndim=ndim, mu_fact=mu_fact, eps_q16=eps_q16,
                        max_iter=max_iter, solver="maxflow")
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        p.stream = ctypes.c_void_p(stream) if stream else None
        self.params = p
        self.n = int(np.prod([int(d) for d in dims]))
        self.n_labels = int(n_labels)
        m = ctypes.c_void_p()
        st = N.dope_ml_create(ctypes.byref(p), int(n_labels), ctypes.byref(m))
        if st != N.DOPE_OK:
            raise N.DopeError(st, N.dope_last_error(None).decode())
        self.m = m

    @classmethod
    def from_problem(cls, mp, **kw):
        t = mp.template
        return cls(t.dims, t.conn, t.block, t.overlap, t.mu0, mp.n_labels, ndim=t.ndim, mu_fact=(t.mu_num, t.mu_den),
                   eps_q16=t.eps_q16, max_iter=t.max_iter, **kw)

    def _check(self, st):
        if st != N.DOPE_OK:
            raise N.DopeError(st, N.dope_ml_last_error(self.m).decode())

    def set_energy(self, D, V):
        Dc = np.ascontiguousarray(D, np.int32) if isinstance(D, np.ndarray) else D
        Vc = np.ascontiguousarray(V, np.int32) if isinstance(V, np.ndarray) else V
        pd, kd = _ptr(Dc)
        pv, kv = _ptr(Vc)
        if kd != kv:
            raise ValueError("D and V must live in the same memory")
        self._check(N.dope_ml_set_energy(self.m, pd, pv, kd))   # copies synchronously

    def step(self, label):
        acc = ctypes.c_int32()
        e = ctypes.c_int64()
        self._check(N.dope_ml_step(self.m, int(label), ctypes.byref(acc), ctypes.byref(e)))
        return acc.value, e.value

    def solve(self, max_cycles=5):
        info = N.dope_ml_info()
        self._check(N.dope_ml_solve(self.m, int(max_cycles), ctypes.byref(info)))
        return _ml_info(info)

    def info(self):
        info = N.dope_ml_info()
        self._check(N.dope_ml_info_get(self.m, ctypes.byref(info)))
        return _ml_info(info)

    def labels(self, out=None):
        if out is None:
            out = np.zeros(self.n, dtype=np.uint8)
        p, k = _ptr(out)
        self._check(N.dope_ml_labels(self.m, p, k))
        return out

    def close(self):
        if getattr(self, "m", None):
            N.dope_ml_destroy(self.m)
            self.m = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()


def _ml_info(info):
    return {"cycles": info.cycles, "moves": info.moves, "accepted": info.accepted,
            "binary_iterations": info.binary_iterations, "energy": info.energy}
