"""ctypes binding of libtcf (argument marshalling only).

Every function here forwards to the C entry point of the same name in
``libtcf.so``; no step of the solver runs in Python.  Loading fails loudly
when the library has not been built.  PyTorch, when present, is used only to
hand a HIP stream (``torch.cuda.current_stream().cuda_stream``) or a device
pointer to the library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TCF_LIB names another build of the same library (e.g. a variant under test)
LIB_PATH = os.environ.get("TCF_LIB", os.path.join(HERE, "libtcf.so"))

TCF_OK, TCF_EINVAL, TCF_ENOMEM, TCF_ENOTSPD, TCF_ENOCONV, TCF_EHIP, TCF_ESTATE = 0, -1, -2, -3, -4, -5, -6
TCF_FP64, TCF_FP32_IR, TCF_FP32_FULL_IR = 0, 1, 2
PRECISIONS = {"fp64": TCF_FP64, "fp32_ir": TCF_FP32_IR, "fp32_full_ir": TCF_FP32_FULL_IR}
(TCF_TOPO_COUNTS, TCF_TOPO_DIRICHLET, TCF_TOPO_TREE_I, TCF_TOPO_TREE_GAMMA, TCF_TOPO_PRIMAL,
 TCF_TOPO_DUAL, TCF_TOPO_INTERIOR, TCF_TOPO_MULT, TCF_TOPO_N, TCF_TOPO_LOOP,
 TCF_TOPO_LOOP_PSI, TCF_TOPO_LOOP_PLAN, TCF_TOPO_COARSE) = range(13)

EXPORTS = ["tcf_default_options", "tcf_last_error", "tcf_create", "tcf_footprint", "tcf_setup",
           "tcf_step", "tcf_step_noalloc", "tcf_sync", "tcf_get_field", "tcf_get_topology", "tcf_get_cond_est",
           "tcf_get_stats",
           "tcf_get_step_log", "tcf_get_state", "tcf_set_state", "tcf_profile_enable",
           "tcf_profile_get", "tcf_profile_get_flops", "tcf_copy_probe", "tcf_bandwidth_probe", "tcf_destroy", "tcf_server_create", "tcf_server_submit",
           "tcf_server_poll", "tcf_server_wait", "tcf_server_fetch", "tcf_server_stats",
           "tcf_server_error", "tcf_server_destroy"]
TCF_REQ_QUEUED, TCF_REQ_RUNNING, TCF_REQ_DONE, TCF_REQ_FAILED = range(4)
KERNEL_GROUPS = ["apply", "precond", "phi", "coarse", "condense", "recover"]

PHI_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double), C.c_int32,
                     C.POINTER(C.c_double), C.c_int32, C.c_int32, C.POINTER(C.c_double),
                     C.c_void_p)

VEC_FN = C.CFUNCTYPE(None, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                     C.c_int32, C.POINTER(C.c_double), C.c_int32, C.c_int32,
                     C.POINTER(C.c_double), C.c_void_p)


class tcf_problem_desc(C.Structure):
    _fields_ = [("np", C.c_int32 * 3),
                ("breaks", C.POINTER(C.c_double) * 3),
                ("nel", C.POINTER(C.c_int32) * 3),
                ("deg", C.POINTER(C.c_int32) * 3),
                ("sigma", C.POINTER(C.c_double)),
                ("nu", C.POINTER(C.c_double)),
                ("src_mask", C.POINTER(C.c_uint8)),
                ("n_rhs", C.c_int32),
                ("phi", PHI_FN),
                ("phi_ctx", C.c_void_p),
                ("amp", C.POINTER(C.c_double)),
                ("dt", C.c_double),
                ("n_steps", C.c_int32),
                ("jvol", VEC_FN),
                ("ainit", VEC_FN),
                ("vec_ctx", C.c_void_p)]


class tcf_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int32),
                ("ir_rtol", C.c_double), ("ir_maxit", C.c_int32), ("check_every", C.c_int32),
                ("use_graph", C.c_int32), ("rhs_batch", C.c_int32), ("pcg_warm", C.c_int32),
                ("precond_scaling", C.c_int32), ("coarse_mode", C.c_int32),
                ("setup_group_mb", C.c_int32), ("panel_chunk", C.c_int32),
                ("autotune", C.c_int32), ("tune_table", C.c_char_p),
                ("deterministic", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class tcf_allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


def torch_allocator():
    """A tcf_allocator that takes the handle's device memory from PyTorch's
    caching allocator (on the stream of each call) and gives it back there.
    Returns (struct, keep-alive list); keep both for the handle's lifetime."""
    import torch

    def _alloc(ctx, nbytes, stream):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0)))
        except RuntimeError:
            return None

    def _free(ctx, ptr, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    return tcf_allocator(None, fa, ff), [fa, ff]


class tcf_stats(C.Structure):
    _fields_ = [("n_patches", C.c_int64), ("n_edges", C.c_int64), ("n_kept", C.c_int64),
                ("n_lambda", C.c_int64), ("n_primal", C.c_int64), ("n_tree_I", C.c_int64),
                ("steps_done", C.c_int32), ("last_pcg_iters", C.c_int32),
                ("total_pcg_iters", C.c_int64), ("max_pcg_iters", C.c_int32),
                ("last_ir_sweeps", C.c_int32), ("nonconverged_steps", C.c_int32),
                ("fail_patch", C.c_int32), ("last_rel_residual", C.c_double),
                ("last_ir_residual", C.c_double), ("setup_ms", C.c_double),
                ("step_ms_total", C.c_double), ("device_bytes", C.c_size_t),
                ("setup_flops", C.c_double), ("cond_est_max", C.c_double),
                ("cond_est_patch", C.c_int32), ("coarse_nodes", C.c_int32),
                ("coarse_launches", C.c_int32), ("coarse_root", C.c_int32),
                ("setup_chunks", C.c_int32), ("coarse_bytes", C.c_double),
                ("device_bytes_peak", C.c_size_t), ("rhs_batch", C.c_int32),
                ("panel_jobs", C.c_int32), ("panel_chunk", C.c_int32 * 4),
                ("panel_chunk_src", C.c_int32), ("panel_tune_us", C.c_double * 20)]


class tcf_server_report(C.Structure):
    _fields_ = [("submitted", C.c_int32), ("admitted", C.c_int32), ("completed", C.c_int32),
                ("failed", C.c_int32), ("running", C.c_int32), ("queued", C.c_int32),
                ("steps", C.c_int64), ("p50_step_ms", C.c_double), ("p99_step_ms", C.c_double),
                ("p50_queue_ms", C.c_double), ("p99_queue_ms", C.c_double),
                ("busy_ms", C.c_double), ("peak_bytes", C.c_size_t)]


_lib = None


def lib():
    """Load libtcf.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_23446_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.tcf_default_options.argtypes = [C.POINTER(tcf_options)]
    L.tcf_default_options.restype = None
    L.tcf_last_error.argtypes = [P]
    L.tcf_last_error.restype = C.c_char_p
    L.tcf_create.argtypes = [C.POINTER(tcf_problem_desc), C.POINTER(tcf_options),
                             C.POINTER(tcf_allocator), C.POINTER(P)]
    L.tcf_footprint.argtypes = [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    L.tcf_setup.argtypes = [P, P]
    L.tcf_step.argtypes = [P, C.c_int32, P]
    L.tcf_step_noalloc.argtypes = [P, C.c_int32, P]
    L.tcf_sync.argtypes = [P, P]
    L.tcf_get_field.argtypes = [P, C.c_int32, P, C.c_size_t, C.c_int32, P]
    L.tcf_get_topology.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
    L.tcf_get_stats.argtypes = [P, C.POINTER(tcf_stats)]
    L.tcf_get_step_log.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double)]
    L.tcf_get_state.argtypes = [P, P, C.POINTER(C.c_size_t), P]
    L.tcf_set_state.argtypes = [P, P, C.c_size_t, P]
    L.tcf_profile_enable.argtypes = [P, C.c_int32]
    L.tcf_profile_get.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_double)]
    L.tcf_profile_get_flops.argtypes = [P, C.c_int32, C.POINTER(C.c_double)]
    L.tcf_copy_probe.argtypes = [C.c_size_t, P]
    L.tcf_bandwidth_probe.argtypes = [C.c_size_t, P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.tcf_destroy.argtypes = [P]
    L.tcf_destroy.restype = None
    L.tcf_server_create.argtypes = [C.c_size_t, C.c_int32, C.POINTER(P)]
    L.tcf_server_submit.argtypes = [P, C.POINTER(tcf_problem_desc), C.POINTER(tcf_options),
                                    C.POINTER(C.c_int32)]
    L.tcf_server_poll.argtypes = [P, C.c_int32, C.POINTER(C.c_int32)]
    L.tcf_server_wait.argtypes = [P, C.c_int32]
    L.tcf_server_fetch.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t, C.POINTER(tcf_stats)]
    L.tcf_server_stats.argtypes = [P, C.POINTER(tcf_server_report)]
    L.tcf_server_error.argtypes = [P, C.c_int32]
    L.tcf_server_error.restype = C.c_char_p
    L.tcf_server_destroy.argtypes = [P]
    L.tcf_server_destroy.restype = None
    for n in EXPORTS:
        if n not in ("tcf_default_options", "tcf_last_error", "tcf_destroy", "tcf_server_destroy",
                     "tcf_server_error"):
            getattr(L, n).restype = C.c_int
    _lib = L
    return L


class TcfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtcf status {code}: {msg}")
        self.code = code


def _dptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def default_options(**kw) -> tcf_options:
    o = tcf_options()
    lib().tcf_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def marshal(prob, precision=None, pcg_rtol=None, pcg_maxit=0, ir_rtol=None, check_every=8,
            use_graph=1, rhs_batch=0, pcg_warm=0, precond_scaling=0, coarse_mode=0,
            setup_group_mb=0, panel_chunk=0, autotune=0, tune_table=None, deterministic=0):
    """(desc, options, keep-alive list) for a workloads.Problem."""
    keep = []
    d = tcf_problem_desc()
    for a in range(3):
        d.np[a] = int(prob.np[a])
        br = np.ascontiguousarray(prob.breaks[a], dtype=np.float64)
        ne = np.ascontiguousarray(prob.nel[a], dtype=np.int32)
        dg = np.ascontiguousarray(prob.deg[a], dtype=np.int32)
        keep += [br, ne, dg]
        d.breaks[a] = _dptr(br, C.c_double)
        d.nel[a] = _dptr(ne, C.c_int32)
        d.deg[a] = _dptr(dg, C.c_int32)
    sig = np.ascontiguousarray(prob.sigma, dtype=np.float64)
    nu = np.ascontiguousarray(prob.nu, dtype=np.float64)
    src = np.ascontiguousarray(prob.src_mask, dtype=np.uint8)
    amp = np.ascontiguousarray(prob.amp, dtype=np.float64)
    keep += [sig, nu, src, amp]
    d.sigma = _dptr(sig, C.c_double)
    d.nu = _dptr(nu, C.c_double)
    d.src_mask = _dptr(src, C.c_uint8)
    d.n_rhs = int(amp.shape[0])
    phi = prob.phi

    def _cb(xs, nx, ys, ny, zs, nz, k, out, ctx):
        x = np.ctypeslib.as_array(xs, shape=(nx,))
        y = np.ctypeslib.as_array(ys, shape=(ny,))
        z = np.ctypeslib.as_array(zs, shape=(nz,))
        v = np.asarray(phi(x, y, z, int(k)), dtype=np.float64).reshape(nx, ny, nz)
        o = np.ctypeslib.as_array(out, shape=(nx * ny * nz,))
        o[:] = v.ravel(order="F")

    if phi is not None:
        cb = PHI_FN(_cb)
        keep.append(cb)
        d.phi = cb
    d.phi_ctx = None

    def _vec(fn):
        def _cbv(s, xs, nx, ys, ny, zs, nz, k, out, ctx):
            x = np.ctypeslib.as_array(xs, shape=(nx,))
            y = np.ctypeslib.as_array(ys, shape=(ny,))
            z = np.ctypeslib.as_array(zs, shape=(nz,))
            v = np.asarray(fn(int(s), x, y, z, int(k)), dtype=np.float64).reshape(nx, ny, nz, 3)
            o = np.ctypeslib.as_array(out, shape=(3 * nx * ny * nz,))
            o[:] = v.transpose(2, 1, 0, 3).ravel()  # component fastest, then x, y, z
        cbv = VEC_FN(_cbv)
        keep.append(cbv)
        return cbv

    if getattr(prob, "jvol", None) is not None:
        d.jvol = _vec(prob.jvol)
    if getattr(prob, "ainit", None) is not None:
        d.ainit = _vec(prob.ainit)
    d.vec_ctx = None
    d.amp = _dptr(amp, C.c_double)
    d.dt = float(prob.dt)
    d.n_steps = int(amp.shape[1])
    prec = precision if precision is not None else prob.precision
    o = default_options(
        precision=PRECISIONS[prec] if isinstance(prec, str) else int(prec),
        pcg_rtol=float(pcg_rtol if pcg_rtol is not None else prob.pcg_rtol),
        pcg_maxit=int(pcg_maxit), ir_rtol=float(ir_rtol if ir_rtol is not None else prob.ir_rtol),
        check_every=int(check_every), use_graph=int(use_graph), rhs_batch=int(rhs_batch),
        pcg_warm=int(pcg_warm), precond_scaling=int(precond_scaling),
        coarse_mode=int(coarse_mode), setup_group_mb=int(setup_group_mb),
        panel_chunk=int(panel_chunk), autotune=int(autotune), deterministic=int(deterministic))
    if tune_table is not None:
        tt = os.fsencode(tune_table)
        keep.append(tt)
        o.tune_table = tt
    return d, o, keep


def tcf_copy_probe(nbytes, stream=None):
    """One launch of the plain copy kernel (traffic-counter reference)."""
    rc = lib().tcf_copy_probe(int(nbytes), Problem._stream(stream))
    if rc != TCF_OK:
        raise TcfError(rc, "tcf_copy_probe")


def _fields_dict(s):
    """A ctypes structure as a dict (arrays as lists)."""
    out = {}
    for f, _ in type(s)._fields_:
        v = getattr(s, f)
        out[f] = list(v) if isinstance(v, C.Array) else v
    return out


def tcf_bandwidth_probe(nbytes, stream=None):
    """(read GB/s, copy GB/s): the device's practical HBM ceilings."""
    r, c = C.c_double(), C.c_double()
    rc = lib().tcf_bandwidth_probe(int(nbytes), Problem._stream(stream), C.byref(r), C.byref(c))
    if rc != TCF_OK:
        raise TcfError(rc, "tcf_bandwidth_probe")
    return r.value, c.value


class Server:
    """Owns one tcf_server (admission by device memory, overlapping requests)."""

    def __init__(self, max_bytes, max_slots):
        self.s = C.c_void_p()
        rc = lib().tcf_server_create(int(max_bytes), int(max_slots), C.byref(self.s))
        if rc != TCF_OK:
            raise TcfError(rc, "tcf_server_create failed")
        self._keep = {}

    def tcf_server_submit(self, prob, **kw):
        d, o, keep = marshal(prob, **kw)
        rid = C.c_int32(-1)
        rc = lib().tcf_server_submit(self.s, C.byref(d), C.byref(o), C.byref(rid))
        # a description that tcf_create rejects gets no id; the callbacks of
        # an admitted request must outlive its worker's setup
        if rid.value >= 0:
            self._keep[rid.value] = (d, o, keep, prob)
        if rc != TCF_OK:
            raise TcfError(rc, lib().tcf_last_error(None).decode())
        return rid.value

    def tcf_server_poll(self, rid):
        st = C.c_int32()
        rc = lib().tcf_server_poll(self.s, int(rid), C.byref(st))
        if rc != TCF_OK:
            raise TcfError(rc, "poll")
        return st.value

    def tcf_server_wait(self, rid):
        return lib().tcf_server_wait(self.s, int(rid))

    def tcf_server_fetch(self, rid, k=0, n_edges=None):
        st = tcf_stats()
        rc = lib().tcf_server_fetch(self.s, int(rid), 0, None, 0, C.byref(st))
        if rc != TCF_OK:
            raise TcfError(rc, "fetch")
        n = int(st.n_edges)
        out = np.zeros(n, dtype=np.float64)
        rc = lib().tcf_server_fetch(self.s, int(rid), int(k), out.ctypes.data_as(C.c_void_p), n,
                                    None)
        if rc != TCF_OK:
            raise TcfError(rc, "fetch")
        return out, _fields_dict(st)

    def tcf_server_error(self, rid):
        return lib().tcf_server_error(self.s, int(rid)).decode()

    def tcf_server_stats(self):
        s = tcf_server_report()
        lib().tcf_server_stats(self.s, C.byref(s))
        return {f: getattr(s, f) for f, _ in tcf_server_report._fields_}

    def tcf_server_destroy(self):
        if getattr(self, "s", None):
            lib().tcf_server_destroy(self.s)
            self.s = None
            self._keep.clear()

    def __del__(self):
        try:
            self.tcf_server_destroy()
        except Exception:
            pass


class Problem:
    """Owns one tcf_problem handle.  Keeps the marshalled arrays and the
    source callback alive for the handle's lifetime (the callback is used
    again by tcf_setup)."""

    def __init__(self, prob, precision=None, pcg_rtol=None, pcg_maxit=0, ir_rtol=None,
                 check_every=8, use_graph=1, rhs_batch=0, pcg_warm=0, precond_scaling=0,
                 coarse_mode=0, setup_group_mb=0, allocator=None, panel_chunk=0, autotune=0,
                 tune_table=None, deterministic=0):
        L = lib()
        self.prob = prob
        d, o, self._keep = marshal(prob, precision, pcg_rtol, pcg_maxit, ir_rtol, check_every,
                                   use_graph, rhs_batch, pcg_warm, precond_scaling, coarse_mode,
                                   setup_group_mb, panel_chunk, autotune, tune_table,
                                   deterministic)
        self._desc = d
        self.opts = o
        # allocator: None (stream-ordered HIP allocation) or a (tcf_allocator,
        # keep-alive) pair such as torch_allocator() returns
        self._alloc = allocator
        h = C.c_void_p()
        rc = L.tcf_create(C.byref(d), C.byref(o),
                          C.byref(allocator[0]) if allocator is not None else None, C.byref(h))
        if rc != TCF_OK:
            raise TcfError(rc, L.tcf_last_error(None).decode())
        self.h = h

    # --- marshalling helpers -------------------------------------------------
    def _check(self, rc, ok=(TCF_OK,)):
        if rc not in ok:
            raise TcfError(rc, lib().tcf_last_error(self.h).decode())
        return rc

    @staticmethod
    def _stream(stream):
        if stream is None:
            return None
        if isinstance(stream, int):
            return C.c_void_p(stream)
        return C.c_void_p(int(stream.cuda_stream))

    # --- entry points --------------------------------------------------------
    def tcf_footprint(self):
        a, b = C.c_size_t(), C.c_size_t()
        self._check(lib().tcf_footprint(self.h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def tcf_setup(self, stream=None):
        return self._check(lib().tcf_setup(self.h, self._stream(stream)))

    def tcf_step(self, nsteps, stream=None, allow_noconv=False):
        ok = (TCF_OK, TCF_ENOCONV) if allow_noconv else (TCF_OK,)
        return self._check(lib().tcf_step(self.h, int(nsteps), self._stream(stream)), ok)

    def tcf_step_noalloc(self, nsteps, stream=None, allow_noconv=False):
        ok = (TCF_OK, TCF_ENOCONV) if allow_noconv else (TCF_OK,)
        return self._check(lib().tcf_step_noalloc(self.h, int(nsteps), self._stream(stream)), ok)

    def tcf_sync(self, stream=None):
        return self._check(lib().tcf_sync(self.h, self._stream(stream)))

    def tcf_get_field(self, k=0, out=None, stream=None):
        """Global edge vector of excitation k.  ``out`` may be a host numpy
        array, or a torch CUDA tensor (filled on the device)."""
        n = self.counts()["n_edges"]
        if out is None:
            out = np.zeros(n, dtype=np.float64)
        if isinstance(out, np.ndarray):
            assert out.dtype == np.float64 and out.size >= n and out.flags.c_contiguous
            self._check(lib().tcf_get_field(self.h, int(k), out.ctypes.data_as(C.c_void_p),
                                            out.size, 0, self._stream(stream)))
        else:  # torch tensor on the GPU
            assert out.is_cuda and out.numel() >= n and str(out.dtype) == "torch.float64"
            self._check(lib().tcf_get_field(self.h, int(k), C.c_void_p(out.data_ptr()),
                                            out.numel(), 1, self._stream(stream)))
        return out

    def tcf_get_topology(self, kind):
        n = C.c_size_t()
        self._check(lib().tcf_get_topology(self.h, int(kind), None, C.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int64)
        n2 = C.c_size_t(out.size)
        self._check(lib().tcf_get_topology(self.h, int(kind), _dptr(out, C.c_int64), C.byref(n2)))
        return out[:n2.value]

    def tcf_get_cond_est(self):
        """Per-patch pivot-ratio condition estimates (after setup)."""
        n = C.c_size_t()
        self._check(lib().tcf_get_cond_est(self.h, None, C.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.float64)
        n2 = C.c_size_t(out.size)
        self._check(lib().tcf_get_cond_est(self.h, _dptr(out, C.c_double), C.byref(n2)))
        return out[:n2.value]

    def tcf_get_stats(self):
        s = tcf_stats()
        self._check(lib().tcf_get_stats(self.h, C.byref(s)))
        return _fields_dict(s)

    def tcf_get_step_log(self, n):
        it = np.zeros(max(n, 1), np.int32)
        ir = np.zeros(max(n, 1), np.int32)
        ms = np.zeros(max(n, 1), np.float64)
        self._check(lib().tcf_get_step_log(self.h, int(n), _dptr(it, C.c_int32), _dptr(ir, C.c_int32),
                                           _dptr(ms, C.c_double)))
        return it[:n], ir[:n], ms[:n]

    def tcf_get_state(self, stream=None):
        n = C.c_size_t()
        self._check(lib().tcf_get_state(self.h, None, C.byref(n), self._stream(stream)))
        buf = np.zeros(n.value, dtype=np.uint8)
        self._check(lib().tcf_get_state(self.h, buf.ctypes.data_as(C.c_void_p), C.byref(n),
                                        self._stream(stream)))
        return buf

    def tcf_set_state(self, buf, stream=None):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        return self._check(lib().tcf_set_state(self.h, buf.ctypes.data_as(C.c_void_p), buf.size,
                                               self._stream(stream)))

    def tcf_profile_enable(self, on=True):
        return self._check(lib().tcf_profile_enable(self.h, int(bool(on))))

    def tcf_profile_get(self):
        """{group: (total_ms, launches, algorithmic bytes per launch)}"""
        out = {}
        for g, name in enumerate(KERNEL_GROUPS):
            ms, n, b = C.c_double(), C.c_int64(), C.c_double()
            self._check(lib().tcf_profile_get(self.h, g, C.byref(ms), C.byref(n), C.byref(b)))
            out[name] = (ms.value, n.value, b.value)
        return out

    def tcf_profile_get_flops(self):
        """{group: algorithmic flops per launch}"""
        out = {}
        for g, name in enumerate(KERNEL_GROUPS):
            f = C.c_double()
            self._check(lib().tcf_profile_get_flops(self.h, g, C.byref(f)))
            out[name] = f.value
        return out

    def tcf_destroy(self):
        if getattr(self, "h", None):
            lib().tcf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.tcf_destroy()
        except Exception:
            pass

    # --- convenience ---------------------------------------------------------
    def counts(self):
        c = self.tcf_get_topology(TCF_TOPO_COUNTS)
        keys = ["n_edges", "n_nodes", "n_vertices_H", "n_plain", "n_floating", "n_lambda",
                "n_primal", "n_kept"]
        return dict(zip(keys, (int(v) for v in c)))
