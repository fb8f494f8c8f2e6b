"""Python binding of libkrps (exact Khatri-Rao leverage-score sampling and
sketched CP-ALS on MI355X).

Argument marshalling only: device memory comes from torch tensors, every
computation runs in the library's HIP kernels.  Loading fails loudly when
the compiled library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkrps.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "krps.h")

KRPS_OK = 0
STATUS = {0: "KRPS_OK", -1: "KRPS_EINVAL", -2: "KRPS_EWORKSPACE", -3: "KRPS_EDEVICE",
          -4: "KRPS_EZERO", -5: "KRPS_ENUMERIC", -6: "KRPS_EUNSUPPORTED"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x2": 2}

_lib = None


class KrpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class TreeInfo(ctypes.Structure):
    _fields_ = [("I", ctypes.c_int64), ("L", ctypes.c_int64), ("F", ctypes.c_int32),
                ("D", ctypes.c_int32), ("n_nodes", ctypes.c_int64), ("tri", ctypes.c_int64),
                ("nodes", ctypes.c_void_p), ("gram", ctypes.c_void_p),
                ("elem_bytes", ctypes.c_int)]


class DrawLayout(ctypes.Structure):
    _fields_ = [("gplus", ctypes.c_size_t), ("rank", ctypes.c_size_t), ("ggt", ctypes.c_size_t),
                ("lam", ctypes.c_size_t), ("vecs", ctypes.c_size_t), ("etree", ctypes.c_size_t),
                ("n_enodes", ctypes.c_int64), ("etree_stride", ctypes.c_int64)]


class Tune(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int32), ("lps", ctypes.c_int32), ("team", ctypes.c_int32),
                ("build_ms", ctypes.c_double), ("draw_ms", ctypes.c_double),
                ("from_cache", ctypes.c_int32)]


class Region(ctypes.Structure):
    _fields_ = [("workspace", ctypes.c_int32), ("name", ctypes.c_char * 28),
                ("offset", ctypes.c_uint64), ("bytes", ctypes.c_uint64), ("need", ctypes.c_uint64)]


class SolveLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_size_t) for n in ("idx", "prob", "w", "rows", "M", "Mp", "Y", "draw",
                                               "yrows", "nyrows", "expanded")]


class Peaks(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("hbm_copy_gbs", "f64_vector_tflops",
                                               "f32_vector_tflops", "f64_matrix_tflops",
                                               "bf16_matrix_tflops")]


def declared_symbols():
    """Function names declared in include/krps.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(krps_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded libkrps (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libkrps.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    c = ctypes
    P = c.c_void_p
    sig = {
        "krps_last_error": (c.c_char_p, []),
        "krps_version": (c.c_char_p, []),
        "krps_ctx_create": (c.c_int, [c.c_int, P, c.POINTER(P)]),
        "krps_ctx_destroy": (c.c_int, [P]),
        "krps_ctx_sync": (c.c_int, [P]),
        "krps_sampler_workspace_bytes": (c.c_int, [c.c_int, c.POINTER(c.c_int64), c.c_int, c.c_int,
                                                   c.c_int, c.POINTER(c.c_size_t)]),
        "krps_sampler_create": (c.c_int, [P, c.c_int, c.POINTER(c.c_int64), c.c_int, c.c_int,
                                          c.POINTER(P), c.c_int, P, c.c_size_t, c.POINTER(P)]),
        "krps_sampler_refresh": (c.c_int, [P, c.c_int]),
        "krps_sampler_destroy": (c.c_int, [P]),
        "krps_sample_workspace_bytes": (c.c_int, [P, c.POINTER(c.c_size_t)]),
        "krps_sample": (c.c_int, [P, c.c_int, c.c_int64, P, P, P, P, P, c.c_size_t, c.c_int]),
        "krps_sample_prepare": (c.c_int, [P, c.c_int, P, c.c_size_t]),
        "krps_sample_seeded": (c.c_int, [P, c.c_int, c.c_int64, c.c_uint64, c.c_uint64, P, P, P,
                                         P, c.c_size_t]),
        "krps_sample_batched_workspace_bytes": (c.c_int, [P, c.c_int, P, P,
                                                          c.POINTER(c.c_size_t)]),
        "krps_sample_batched": (c.c_int, [P, c.c_int, P, P, P, P, P, P, P, c.c_size_t]),
        "krps_sample_batched_prepare": (c.c_int, [P, c.c_int, P, P, P, c.c_size_t]),
        "krps_sample_batched_draw": (c.c_int, [P, c.c_int, P, P, P, P, P, P, P, c.c_size_t]),
        "krps_sample_draw": (c.c_int, [P, c.c_int, c.c_int64, P, P, P, P, P, c.c_size_t]),
        "krps_row_prob": (c.c_int, [P, c.c_int, c.c_int64, P, P, P, c.c_size_t]),
        "krps_tensor_workspace_bytes": (c.c_int, [c.c_int, c.POINTER(c.c_int64), c.c_int64,
                                                  c.POINTER(c.c_size_t)]),
        "krps_tensor_create": (c.c_int, [P, c.c_int, c.POINTER(c.c_int64), c.c_int64, P, P, P,
                                         c.c_size_t, c.POINTER(P)]),
        "krps_tensor_destroy": (c.c_int, [P]),
        "krps_tensor_norm2": (c.c_int, [P, c.POINTER(c.c_double)]),
        "krps_sampler_set_lps": (c.c_int, [P, c.c_int]),
        "krps_init_range_finder": (c.c_int, [P, P, c.c_int, c.c_uint64, P, P, c.c_size_t]),
        "krps_autotune_workspace_bytes": (c.c_int, [c.c_int, c.POINTER(c.c_int64), c.c_int,
                                                    c.c_int, c.c_int64, c.POINTER(c.c_size_t)]),
        "krps_autotune": (c.c_int, [P, c.c_int, c.POINTER(c.c_int64), c.c_int, c.c_int,
                                    c.POINTER(P), c.c_int64, P, P, c.c_size_t, c.c_char_p,
                                    c.POINTER(Tune)]),
        "krps_lstsq_workspace_bytes": (c.c_int, [c.c_int, c.c_int64, c.c_int64,
                                                 c.POINTER(c.c_size_t)]),
        "krps_sketched_lstsq": (c.c_int, [P, c.c_int, c.c_int64, P, P, c.c_int64, P, P, c.c_int,
                                          P, c.c_size_t]),
        "krps_tensor_stored_entries": (c.c_int, [P, c.POINTER(c.c_int64)]),
        "krps_tensor_hot_rows": (c.c_int, [P, c.c_int, c.POINTER(c.c_int32), c.POINTER(c.c_int)]),
        "krps_solve_workspace_bytes": (c.c_int, [P, P, c.c_int64, c.POINTER(c.c_size_t)]),
        "krps_solve_layout_query": (c.c_int, [P, P, c.c_int64, c.POINTER(SolveLayout)]),
        "krps_normalize_factor": (c.c_int, [P, c.c_int, P, P, c.c_size_t]),
        "krps_sketched_solve": (c.c_int, [P, P, c.c_int, c.c_int64, P, P, P, c.c_size_t]),
        "krps_als_sweep": (c.c_int, [P, P, c.c_int64, P, P, P, c.c_size_t, c.c_int]),
        "krps_fit": (c.c_int, [P, P, P, c.POINTER(c.c_double), P, c.c_size_t]),
        "krps_sampler_tree_info": (c.c_int, [P, c.c_int, c.POINTER(TreeInfo)]),
        "krps_sampler_check": (c.c_int, [P, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]),
        "krps_sampler_set_filter": (c.c_int, [P, c.c_int]),
        "krps_sampler_set_build": (c.c_int, [P, c.c_int]),
        "krps_sampler_set_deterministic": (c.c_int, [P, c.c_int]),
        "krps_sampler_update_entries": (c.c_int, [P, c.c_int, c.c_int64, c.POINTER(c.c_int64),
                                                  c.POINTER(c.c_int32),
                                                  c.POINTER(c.c_double)]),
        "krps_sample_static": (c.c_int, [P, c.c_int, c.c_int64, P, P, P, P]),
        "krps_exact_solve": (c.c_int, [P, P, c.c_int, P, P, c.c_size_t]),
        "krps_measure_peaks": (c.c_int, [P, P, c.c_size_t, c.POINTER(Peaks)]),
        "krps_sketched_solve_seeded": (c.c_int, [P, P, c.c_int, c.c_int64, c.c_uint64,
                                                 c.c_uint64, c.c_uint64, P, P, c.c_size_t]),
        "krps_als_sweep_seeded": (c.c_int, [P, P, c.c_int64, c.c_uint64, c.c_uint64, c.c_uint64,
                                            P, P, c.c_size_t, c.c_int]),
        "krps_sample_batched_seeded": (c.c_int, [P, c.c_int, P, P, P, P, P, P, P, P,
                                                 c.c_size_t]),
        "krps_workspace_regions": (c.c_int, [c.c_int, c.POINTER(c.c_int64), c.c_int, c.c_int,
                                             c.c_int, c.c_int64, c.c_int64, c.POINTER(Region),
                                             c.c_int, c.POINTER(c.c_int)]),
        "krps_draw_layout_query": (c.c_int, [P, c.POINTER(DrawLayout)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(code):
    if code != KRPS_OK:
        raise KrpsError(code, lib().krps_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Context:
    """Device + HIP stream (torch's current stream unless given)."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().krps_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def sync(self):
        check(lib().krps_ctx_sync(self.handle))

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.krps_ctx_destroy(self.handle)
            self.handle = None


def measure_peaks(ctx: "Context", nbytes=1 << 30):
    """Measured HBM copy bandwidth and vector / matrix-core peaks (dict)."""
    torch = ctx.torch
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=ctx.device)
    out = Peaks()
    check(lib().krps_measure_peaks(ctx.handle, _ptr(ws), ws.numel(), ctypes.byref(out)))
    return {n: getattr(out, n) for n, _ in Peaks._fields_}


def workspace_regions(dims, R, F=0, precision="fp32", nnz=1, J=1):
    """Regions of every workspace the library plans (host only): a list of
    dicts with workspace, name, offset, bytes and need."""
    n = len(dims)
    arr = (ctypes.c_int64 * n)(*[int(d) for d in dims])
    cnt = ctypes.c_int()
    check(lib().krps_workspace_regions(n, arr, int(R), int(F), PRECISION[precision], int(nnz),
                                       int(J), None, 0, ctypes.byref(cnt)))
    buf = (Region * cnt.value)()
    check(lib().krps_workspace_regions(n, arr, int(R), int(F), PRECISION[precision], int(nnz),
                                       int(J), buf, cnt.value, ctypes.byref(cnt)))
    return [{"workspace": r.workspace, "name": r.name.decode(), "offset": r.offset,
             "bytes": r.bytes, "need": r.need} for r in buf]


def sampler_workspace_bytes(dims, R, F=0, precision="fp32"):
    n = len(dims)
    arr = (ctypes.c_int64 * n)(*[int(d) for d in dims])
    out = ctypes.c_size_t()
    check(lib().krps_sampler_workspace_bytes(n, arr, int(R), int(F), PRECISION[precision],
                                             ctypes.byref(out)))
    return out.value


class Sampler:
    """Sampler over device factors (Algorithm 1).  ``factors``: list of
    contiguous CUDA tensors ``[I_j, R]`` (float64 for ``fp64``, float32
    otherwise).  The tensors are referenced, not copied."""

    def __init__(self, ctx: Context, factors, precision="fp32", F=0, lps=0, team=0):
        torch = ctx.torch
        self.ctx = ctx
        self.precision = precision
        self.factors = list(factors)
        self.N = len(self.factors)
        self.R = int(self.factors[0].shape[1])
        self.dims = [int(U.shape[0]) for U in self.factors]
        want = torch.float64 if precision == "fp64" else torch.float32
        for U in self.factors:
            if U.dtype != want or not U.is_contiguous() or U.device != ctx.device:
                raise ValueError(f"factors must be contiguous {want} tensors on {ctx.device}")
        nbytes = sampler_workspace_bytes(self.dims, self.R, F, precision)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=ctx.device)
        arr = (ctypes.c_int64 * self.N)(*self.dims)
        ptrs = (ctypes.c_void_p * self.N)(*[U.data_ptr() for U in self.factors])
        h = ctypes.c_void_p()
        check(lib().krps_sampler_create(ctx.handle, self.N, arr, self.R, int(F), ptrs,
                                        PRECISION[precision], _ptr(self.ws), nbytes,
                                        ctypes.byref(h)))
        self.handle = h
        self.deterministic = False
        if lps:
            check(lib().krps_sampler_set_lps(self.handle, int(lps)))
        if team:
            # the trees were built with the default team at creation; the
            # nodes do not depend on it, later rebuilds use this one
            check(lib().krps_sampler_set_build(self.handle, int(team)))
        sz = ctypes.c_size_t()
        check(lib().krps_sample_workspace_bytes(self.handle, ctypes.byref(sz)))
        self.draw_ws = torch.empty(sz.value, dtype=torch.uint8, device=ctx.device)

    def refresh(self, j):
        check(lib().krps_sampler_refresh(self.handle, int(j)))

    def update_entries(self, j, rows, cols, values):
        """krps_sampler_update_entries: ``U_j[rows[m], cols[m]] := values[m]``
        in order, with the factor tree updated along each row's path
        (host sequences)."""
        M = len(rows)
        ra = (ctypes.c_int64 * M)(*[int(x) for x in rows])
        ca = (ctypes.c_int32 * M)(*[int(x) for x in cols])
        va = (ctypes.c_double * M)(*[float(x) for x in values])
        check(lib().krps_sampler_update_entries(self.handle, int(j), M, ra, ca, va))

    def check_status(self):
        """Reads and clears the device status (raises on a zero product or a
        non-finite value); returns the number of sampled rows since the last
        check whose computed probability was not positive.  The number of
        float64 walks re-walked from the float64 tree since the last check
        is left in ``self.rewalked``."""
        n, r = ctypes.c_int64(), ctypes.c_int64()
        check(lib().krps_sampler_check(self.handle, ctypes.byref(n), ctypes.byref(r)))
        self.rewalked = r.value
        return n.value

    def set_deterministic(self, on=True):
        """Sketched solves sum Y in fixed point (order-independent, so runs
        repeat bit for bit) instead of with float atomics; Y is then float64
        on every path."""
        check(lib().krps_sampler_set_deterministic(self.handle, 1 if on else 0))
        self.deterministic = bool(on)

    def set_filter(self, top):
        """Levels of each factor tree the float64 walk reads from the
        float64 nodes before it decides from their float32 copy (-1: the
        default; >= the depth: the copy is not used)."""
        check(lib().krps_sampler_set_filter(self.handle, int(top)))

    def sample(self, exclude, uniforms, prob=True, rows=False, check_status=False):
        """Draws ``J = uniforms.shape[0]`` samples; returns ``(idx, prob, rows)``."""
        torch = self.ctx.torch
        J = int(uniforms.shape[0])
        dev = self.ctx.device
        idx = torch.empty((J, self.N), dtype=torch.int32, device=dev)
        p = torch.empty(J, dtype=torch.float64, device=dev) if prob else None
        rdt = torch.float64 if self.precision == "fp64" else torch.float32
        r = torch.empty((J, self.R), dtype=rdt, device=dev) if rows else None
        check(lib().krps_sample(self.handle, int(exclude), J, _ptr(uniforms), _ptr(idx), _ptr(p),
                                _ptr(r), _ptr(self.draw_ws), self.draw_ws.numel(),
                                1 if check_status else 0))
        return idx, p, r

    def sample_static(self, exclude, uniforms, idx, prob=None, rows=None):
        """krps_sample into caller tensors with the library's static per-GPU
        scratch instead of a workspace (no allocation in the call)."""
        check(lib().krps_sample_static(self.handle, int(exclude), int(uniforms.shape[0]),
                                       _ptr(uniforms), _ptr(idx), _ptr(prob), _ptr(rows)))

    def sample_seeded(self, exclude, J, seed, ctr_base=0, prob=True):
        """Draws J samples with uniforms generated in the walk (Philox4x64-10
        of (ctr_base + d, k, 0, 0) under (seed, 0)); returns ``(idx, prob)``."""
        torch = self.ctx.torch
        dev = self.ctx.device
        idx = torch.empty((int(J), self.N), dtype=torch.int32, device=dev)
        p = torch.empty(int(J), dtype=torch.float64, device=dev) if prob else None
        check(lib().krps_sample_seeded(self.handle, int(exclude), int(J), ctypes.c_uint64(int(seed)),
                                       ctypes.c_uint64(int(ctr_base)), _ptr(idx), _ptr(p), None,
                                       _ptr(self.draw_ws), self.draw_ws.numel()))
        return idx, p

    def prepare(self, exclude):
        """The set-up part of Algorithm 2 (before its per-sample loop) for
        ``exclude`` into this sampler's draw workspace."""
        check(lib().krps_sample_prepare(self.handle, int(exclude), _ptr(self.draw_ws),
                                        self.draw_ws.numel()))

    def draw(self, exclude, uniforms, idx, prob=None, rows=None):
        """The walk alone (after :meth:`prepare` with the same ``exclude``),
        into caller-provided output tensors."""
        check(lib().krps_sample_draw(self.handle, int(exclude), int(uniforms.shape[0]),
                                     _ptr(uniforms), _ptr(idx), _ptr(prob), _ptr(rows),
                                     _ptr(self.draw_ws), self.draw_ws.numel()))

    def row_prob(self, exclude, idx):
        torch = self.ctx.torch
        M = int(idx.shape[0])
        p = torch.empty(M, dtype=torch.float64, device=self.ctx.device)
        check(lib().krps_row_prob(self.handle, int(exclude), M, _ptr(idx), _ptr(p),
                                  _ptr(self.draw_ws), self.draw_ws.numel()))
        return p

    def tree_info(self, j):
        ti = TreeInfo()
        check(lib().krps_sampler_tree_info(self.handle, int(j), ctypes.byref(ti)))
        return ti

    def tree_nodes(self, j):
        """Copy of the stored nodes of factor tree ``j`` as ``[n_nodes, tri]``."""
        torch = self.ctx.torch
        ti = self.tree_info(j)
        off = ti.nodes - self.ws.data_ptr()
        n = ti.n_nodes * ti.tri * ti.elem_bytes
        dt = torch.float64 if ti.elem_bytes == 8 else torch.float32
        return self.ws[off:off + n].view(dt).view(ti.n_nodes, ti.tri).clone()

    def gram(self, j):
        torch = self.ctx.torch
        ti = self.tree_info(j)
        off = ti.gram - self.ws.data_ptr()
        return self.ws[off:off + self.R * self.R * 8].view(torch.float64).view(self.R, self.R).clone()

    def draw_layout(self):
        dl = DrawLayout()
        check(lib().krps_draw_layout_query(self.handle, ctypes.byref(dl)))
        return dl

    def draw_parts(self, ws=None):
        """Views of what the last sample()/row_prob() prepared (or, with
        ``ws``, the preparation held in that per-draw workspace)."""
        torch = self.ctx.torch
        dl = self.draw_layout()
        R, N = self.R, self.N
        ws = self.draw_ws if ws is None else ws
        tri = R * (R + 1) // 2
        es = 8 if self.precision == "fp64" else 4
        dt = torch.float64 if es == 8 else torch.float32

        def view(off, n, dtype, nb):
            return ws[off:off + n * nb].view(dtype)

        return {
            "gplus": view(dl.gplus, R * R, torch.float64, 8).view(R, R).clone(),
            "rank": int(view(dl.rank, 1, torch.int32, 4).item()),
            "sweeps": view(dl.rank, 2 + N, torch.int32, 4).cpu().numpy()[1:].tolist(),
            "ggt": view(dl.ggt, N * R * R, torch.float64, 8).view(N, R, R).clone(),
            "lam": view(dl.lam, N * R, torch.float64, 8).view(N, R).clone(),
            "vecs": view(dl.vecs, N * R * R, dt, es).view(N, R, R).clone(),
            "etree": view(dl.etree, N * dl.etree_stride, dt, es).view(N, dl.etree_stride)
                     [:, :dl.n_enodes * tri].reshape(N, dl.n_enodes, tri).clone(),
        }

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.krps_sampler_destroy(self.handle)
            self.handle = None


class Batch:
    """Many samplers drawn together (Appendix A.10 batching): batched
    preparations and one persistent walk launch per storage type and shape
    class.  ``excludes[p]`` is the exclusion of ``samplers[p]`` (a sampler
    may appear several times with different exclusions)."""

    def __init__(self, ctx: "Context", samplers, excludes):
        torch = ctx.torch
        self.ctx = ctx
        self.samplers = list(samplers)
        self.P = len(self.samplers)
        self._h = (ctypes.c_void_p * self.P)(*[sp.handle.value for sp in self.samplers])
        self._ex = (ctypes.c_int * self.P)(*[int(e) for e in excludes])
        nb = ctypes.c_size_t()
        check(lib().krps_sample_batched_workspace_bytes(ctx.handle, self.P, self._h, self._ex,
                                                        ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)

    def prepare(self):
        check(lib().krps_sample_batched_prepare(self.ctx.handle, self.P, self._h, self._ex,
                                                _ptr(self.ws), self.ws.numel()))

    def draw(self, uniforms, idx, prob=None):
        """Walks into caller tensors: ``uniforms[p]`` float64 ``[J_p, N_p, 2]``,
        ``idx[p]`` int32 ``[J_p, N_p]``, ``prob[p]`` float64 ``[J_p]`` or None."""
        P = self.P
        Ja = (ctypes.c_int64 * P)(*[int(u.shape[0]) for u in uniforms])
        ua = (ctypes.c_void_p * P)(*[u.data_ptr() for u in uniforms])
        ia = (ctypes.c_void_p * P)(*[i.data_ptr() for i in idx])
        pa = None
        if prob is not None:
            pa = (ctypes.c_void_p * P)(*[(q.data_ptr() if q is not None else 0) for q in prob])
        check(lib().krps_sample_batched_draw(self.ctx.handle, P, self._h, self._ex, Ja, ua, ia,
                                             pa, _ptr(self.ws), self.ws.numel()))

    def sample(self, uniforms, with_prob=True):
        """One krps_sample_batched call; returns ``(idx_list, prob_list)``."""
        torch = self.ctx.torch
        dev = self.ctx.device
        idx = [torch.empty((int(u.shape[0]), sp.N), dtype=torch.int32, device=dev)
               for u, sp in zip(uniforms, self.samplers)]
        prob = [torch.empty(int(u.shape[0]), dtype=torch.float64, device=dev) if with_prob
                else None for u in uniforms]
        P = self.P
        Ja = (ctypes.c_int64 * P)(*[int(u.shape[0]) for u in uniforms])
        ua = (ctypes.c_void_p * P)(*[u.data_ptr() for u in uniforms])
        ia = (ctypes.c_void_p * P)(*[i.data_ptr() for i in idx])
        pa = (ctypes.c_void_p * P)(*[(q.data_ptr() if q is not None else 0) for q in prob])
        check(lib().krps_sample_batched(self.ctx.handle, P, self._h, self._ex, Ja, ua, ia,
                                        pa if with_prob else None, _ptr(self.ws), self.ws.numel()))
        return idx, prob


    def sample_seeded(self, J, seeds, ctr_bases, with_prob=True):
        """krps_sample_batched_seeded: problem p draws ``J[p]`` samples with
        uniforms generated in the walk from ``seeds[p]``, ``ctr_bases[p]``."""
        torch = self.ctx.torch
        dev = self.ctx.device
        P = self.P
        idx = [torch.empty((int(J[p]), sp.N), dtype=torch.int32, device=dev)
               for p, sp in enumerate(self.samplers)]
        prob = [torch.empty(int(J[p]), dtype=torch.float64, device=dev) if with_prob else None
                for p in range(P)]
        Ja = (ctypes.c_int64 * P)(*[int(j) for j in J])
        sa = (ctypes.c_uint64 * P)(*[int(x) for x in seeds])
        ca = (ctypes.c_uint64 * P)(*[int(x) for x in ctr_bases])
        ia = (ctypes.c_void_p * P)(*[i.data_ptr() for i in idx])
        pa = (ctypes.c_void_p * P)(*[(q.data_ptr() if q is not None else 0) for q in prob])
        check(lib().krps_sample_batched_seeded(self.ctx.handle, P, self._h, self._ex, Ja, sa, ca,
                                               ia, pa if with_prob else None, _ptr(self.ws),
                                               self.ws.numel()))
        return idx, prob


def sample_batched(ctx: "Context", samplers, excludes, uniforms, with_prob=True):
    """Algorithm 2 for many samplers in one batched call.  ``uniforms[p]``:
    CUDA float64 ``[J_p, N_p, 2]``.  Returns ``(idx_list, prob_list)``."""
    return Batch(ctx, samplers, excludes).sample(uniforms, with_prob)


def autotune(ctx: "Context", factors, uniforms, precision="fp32", cache_path=None):
    """Leaf size F, walk lanes per sample and tree-build team width for
    these factors: measured (rebuild + draw of J = uniforms.shape[0]
    samples; uniforms float64 ``[J, N, 2]`` on the device) or read from the
    JSON-lines cache.  Returns a dict with F, lps, team, build_ms, draw_ms,
    from_cache."""
    torch = ctx.torch
    N = len(factors)
    R = int(factors[0].shape[1])
    dims = [int(U.shape[0]) for U in factors]
    J = int(uniforms.shape[0])
    arr = (ctypes.c_int64 * N)(*dims)
    nb = ctypes.c_size_t()
    check(lib().krps_autotune_workspace_bytes(N, arr, R, PRECISION[precision], J,
                                              ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
    ptrs = (ctypes.c_void_p * N)(*[U.data_ptr() for U in factors])
    t = Tune()
    check(lib().krps_autotune(ctx.handle, N, arr, R, PRECISION[precision], ptrs, J,
                              _ptr(uniforms), _ptr(ws), ws.numel(),
                              None if cache_path is None else str(cache_path).encode(),
                              ctypes.byref(t)))
    return {"F": t.F, "lps": t.lps, "team": t.team, "build_ms": t.build_ms,
            "draw_ms": t.draw_ms, "from_cache": bool(t.from_cache)}


def sketched_lstsq(ctx: "Context", rows, prob, sb_rows, precision=None):
    """min_X ||S A X - S B||_F from sampled rows ``rows`` [J, R], their
    probabilities ``prob`` [J] (float64) and the sampled rows of B
    ``sb_rows`` [J, n]; returns X [R, n] (float64)."""
    torch = ctx.torch
    J, R = int(rows.shape[0]), int(rows.shape[1])
    n = int(sb_rows.shape[1])
    if precision is None:
        precision = "fp64" if rows.dtype == torch.float64 else "fp32"
    nb = ctypes.c_size_t()
    check(lib().krps_lstsq_workspace_bytes(R, J, n, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
    X = torch.empty((R, n), dtype=torch.float64, device=ctx.device)
    rows, prob, sb_rows = rows.contiguous(), prob.contiguous(), sb_rows.contiguous()
    check(lib().krps_sketched_lstsq(ctx.handle, R, J, _ptr(rows), _ptr(prob), n, _ptr(sb_rows),
                                    _ptr(X), PRECISION[precision], _ptr(ws), ws.numel()))
    return X


class Tensor:
    """Sparse COO tensor with its per-mode fiber index on the device.
    ``idx``: int32 CUDA tensor ``[nnz, N]``, ``val``: float32 ``[nnz]``."""

    def __init__(self, ctx: Context, dims, idx, val):
        torch = ctx.torch
        self.ctx = ctx
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.nnz = int(val.shape[0])
        if idx.dtype != torch.int32 or val.dtype != torch.float32:
            raise ValueError("idx must be int32 and val float32")
        idx = idx.contiguous()
        val = val.contiguous()
        arr = (ctypes.c_int64 * self.N)(*self.dims)
        nb = ctypes.c_size_t()
        check(lib().krps_tensor_workspace_bytes(self.N, arr, self.nnz, ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=ctx.device)
        h = ctypes.c_void_p()
        check(lib().krps_tensor_create(ctx.handle, self.N, arr, self.nnz, _ptr(idx), _ptr(val),
                                       _ptr(self.ws), nb.value, ctypes.byref(h)))
        self.handle = h

    @property
    def norm2(self):
        v = ctypes.c_double()
        check(lib().krps_tensor_norm2(self.handle, ctypes.byref(v)))
        return v.value

    @property
    def stored_entries(self):
        """Distinct coordinates (duplicates are merged into one entry)."""
        v = ctypes.c_int64()
        check(lib().krps_tensor_stored_entries(self.handle, ctypes.byref(v)))
        return v.value

    def hot_rows(self, j):
        """Rows of mode ``j`` with the most stored entries, in decreasing
        count (host int list of at most 512)."""
        buf = (ctypes.c_int32 * 512)()
        n = ctypes.c_int()
        check(lib().krps_tensor_hot_rows(self.handle, int(j), buf, ctypes.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.krps_tensor_destroy(self.handle)
            self.handle = None


class CPALS:
    """Sketched CP-ALS state: a sampler over the factors, a tensor and the
    solve workspace for J samples per solve."""

    def __init__(self, sampler: Sampler, tensor: Tensor, J):
        torch = sampler.ctx.torch
        self.S, self.T, self.J = sampler, tensor, int(J)
        nb = ctypes.c_size_t()
        check(lib().krps_solve_workspace_bytes(sampler.handle, tensor.handle, self.J,
                                               ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=sampler.ctx.device)
        self.sigma = torch.ones(sampler.R, dtype=torch.float64, device=sampler.ctx.device)
        lay = SolveLayout()
        check(lib().krps_solve_layout_query(sampler.handle, tensor.handle, self.J,
                                            ctypes.byref(lay)))
        self.layout = lay

    def normalize(self, j):
        check(lib().krps_normalize_factor(self.S.handle, int(j), _ptr(self.sigma), _ptr(self.ws),
                                          self.ws.numel()))

    def init_range_finder(self, j, seed):
        """U_j = mat(T, j) S with a generated Gaussian sketch, normalised
        (sigma of mode j into self.sigma); Z_j rebuilt."""
        check(lib().krps_init_range_finder(self.S.handle, self.T.handle, int(j),
                                           ctypes.c_uint64(int(seed)), _ptr(self.sigma),
                                           _ptr(self.ws), self.ws.numel()))

    def solve(self, j, uniforms):
        check(lib().krps_sketched_solve(self.S.handle, self.T.handle, int(j), self.J,
                                        _ptr(uniforms), _ptr(self.sigma), _ptr(self.ws),
                                        self.ws.numel()))

    def sweep(self, uniforms, use_graph=False):
        check(lib().krps_als_sweep(self.S.handle, self.T.handle, self.J, _ptr(uniforms),
                                   _ptr(self.sigma), _ptr(self.ws), self.ws.numel(),
                                   1 if use_graph else 0))

    def exact_solve(self, j):
        """The exact ALS step of mode j (full sparse MTTKRP, no sampling)."""
        check(lib().krps_exact_solve(self.S.handle, self.T.handle, int(j), _ptr(self.sigma),
                                     _ptr(self.ws), self.ws.numel()))

    def exact_parts(self, j):
        """M^+ and the MTTKRP (listed rows, float64) of the last exact solve."""
        torch = self.S.ctx.torch
        lay = SolveLayout()
        check(lib().krps_solve_layout_query(self.S.handle, self.T.handle, 1, ctypes.byref(lay)))
        R, ws = self.S.R, self.ws
        n = int(ws[lay.nyrows:lay.nyrows + 8].view(torch.int64).item())
        rows = ws[lay.yrows:lay.yrows + 4 * n].view(torch.int32).clone()
        I = self.S.dims[j]
        full = ws[lay.Y:lay.Y + I * R * 8].view(torch.float64).view(I, R)
        Y = torch.zeros(I, R, dtype=torch.float64, device=full.device)
        Y[rows.long()] = full[rows.long()]
        return {"Mp": ws[lay.Mp:lay.Mp + R * R * 8].view(torch.float64).view(R, R).clone(),
                "Y": Y, "yrows": rows}

    def solve_seeded(self, j, seed, ctr_base, sweep):
        """One solve with in-kernel uniforms (counter word 2 = sweep * N + j)."""
        check(lib().krps_sketched_solve_seeded(self.S.handle, self.T.handle, int(j), self.J,
                                               ctypes.c_uint64(int(seed)),
                                               ctypes.c_uint64(int(ctr_base)),
                                               ctypes.c_uint64(int(sweep)), _ptr(self.sigma),
                                               _ptr(self.ws), self.ws.numel()))

    def sweep_seeded(self, seed, ctr_base, sweep, use_graph=False):
        """One sweep with in-kernel uniforms; a captured graph is replayed for
        every sweep number."""
        check(lib().krps_als_sweep_seeded(self.S.handle, self.T.handle, self.J,
                                          ctypes.c_uint64(int(seed)),
                                          ctypes.c_uint64(int(ctr_base)),
                                          ctypes.c_uint64(int(sweep)), _ptr(self.sigma),
                                          _ptr(self.ws), self.ws.numel(), 1 if use_graph else 0))

    def fit(self):
        v = ctypes.c_double()
        check(lib().krps_fit(self.S.handle, self.T.handle, _ptr(self.sigma), ctypes.byref(v),
                             _ptr(self.ws), self.ws.numel()))
        return v.value

    def parts(self, j):
        """Views of the last solve's pieces (for mode ``j``'s Y height)."""
        torch = self.S.ctx.torch
        l, R, N, J = self.layout, self.S.R, self.S.N, self.J
        ws = self.ws
        es = 8 if self.S.precision == "fp64" else 4
        dt = torch.float64 if es == 8 else torch.float32

        def view(off, n, dtype, nb):
            return ws[off:off + n * nb].view(dtype)

        return {
            "idx": view(l.idx, J * N, torch.int32, 4).view(J, N).clone(),
            "prob": view(l.prob, J, torch.float64, 8).clone(),
            "w": view(l.w, J, torch.float64, 8).clone(),
            "rows": (view(l.rows, J * R, torch.float32, 4) if self.S.precision == "bf16x2"
                     else view(l.rows, J * R, torch.float64, 8)).view(J, R).clone(),
            "M": view(l.M, R * R, torch.float64, 8).view(R, R).clone(),
            "Mp": view(l.Mp, R * R, torch.float64, 8).view(R, R).clone(),
            "Y": self._y(j),
            "yrows": self._yrows(),
            "expanded": view(l.expanded, 1, torch.int64, 8).clone(),
        }

    def draw_parts(self):
        """The preparation of the last solve's draw (G^+, eigenpairs of
        every G_{>k}, eigen-trees, Jacobi sweep counts)."""
        return self.S.draw_parts(self.ws[self.layout.draw:])

    def _yrows(self):
        l, ws = self.layout, self.ws
        n = int(ws[l.nyrows:l.nyrows + 8].view(self.S.ctx.torch.int64).item())
        return ws[l.yrows:l.yrows + 4 * n].view(self.S.ctx.torch.int32).clone()

    def _y(self, j):
        """(S B)^T S A of the last solve: the listed rows from the workspace,
        zero elsewhere."""
        torch = self.S.ctx.torch
        l, R, ws = self.layout, self.S.R, self.ws
        I = self.S.dims[j]
        if self.S.precision == "bf16x2" and not self.S.deterministic:
            full = ws[l.Y:l.Y + I * R * 4].view(torch.float32).view(I, R)
        else:
            full = ws[l.Y:l.Y + I * R * 8].view(torch.float64).view(I, R)
        rows = self._yrows().long()
        Y = torch.zeros(I, R, dtype=torch.float64, device=full.device)
        Y[rows] = full[rows].double()
        return Y
