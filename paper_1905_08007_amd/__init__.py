"""MI355X hot path of Volkov's 5-loop QED AMM method: per-sample evaluation
of the IR/UV-subtracted Feynman-parametric integrand of vertex graphs without
lepton loops, at points from each graph's Hepp-sector PDF, accumulated into
per-graph value and variance sums.

This module is the argument-marshalling layer over the C ABI of
``libqedamm.so`` (declared in ``include/qedamm.h``); every step of the path
runs in the library's HIP kernels.  PyTorch provides device memory and
streams.  Importing succeeds without the library; every call that needs it
raises ``RuntimeError`` when it is missing (there is no CPU fallback).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqedamm.so")

QA_FP64, QA_FP64_BOUND, QA_DD, QA_FP64_EST = 0, 1, 2, 3


class QaGraph(C.Structure):
    _fields_ = [("loops", C.c_int32), ("x", C.c_int32), ("mate", C.c_int8 * 12),
                ("mult", C.c_int32), ("cls", C.c_int32 * 3)]


ACC_DTYPE = np.dtype([("n", "<u8"), ("s1_hi", "<f8"), ("s1_lo", "<f8"), ("s2_hi", "<f8"),
                      ("s2_lo", "<f8"), ("n_flagged", "<u8"), ("n_bad", "<u8"), ("n_residual", "<u8")])
ACC_BYTES = ACC_DTYPE.itemsize  # 64
RESULT_DTYPE = np.dtype([("value", "<f8"), ("sigma", "<f8"), ("mean", "<f8"), ("sd", "<f8"), ("n", "<u8"),
                         ("n_bad", "<u8"), ("n_flagged", "<u8"), ("n_residual", "<u8")])

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1905_08007_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, sz, u64, u32, i32 = C.c_void_p, C.c_size_t, C.c_uint64, C.c_uint32, C.c_int
        L.qa_last_error.restype = C.c_char_p
        L.qa_enumerate_graphs.argtypes = [i32, i32, i32, i32, vp, sz, C.POINTER(sz)]
        L.qa_build_forests.argtypes = [vp, sz, i32, C.POINTER(vp)]
        L.qa_set_destroy.argtypes = [vp]
        L.qa_set_destroy.restype = None
        L.qa_forests_serialize.argtypes = [vp, vp, sz, C.POINTER(sz)]
        L.qa_set_stats.argtypes = [vp, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
        L.qa_pdf_create.argtypes = [vp, vp, C.POINTER(vp)]
        L.qa_pdf_destroy.argtypes = [vp]
        L.qa_pdf_destroy.restype = None
        L.qa_pdf_tables.argtypes = [vp, u32, vp, vp]
        L.qa_pdf_dlogw.argtypes = [vp, u32, vp]
        L.qa_device_bytes.argtypes = [vp, vp, C.POINTER(sz)]
        L.qa_upload.argtypes = [vp, vp, vp, sz, vp]
        L.qa_sample_pdf.argtypes = [vp, u32, u64, u32, u64, u64, vp, vp, vp, vp]
        L.qa_eval_integrand.argtypes = [vp, u32, vp, u64, i32, vp, vp, vp, vp]
        L.qa_accumulate.argtypes = [vp, vp, u64, vp, vp]
        L.qa_work_bytes.argtypes = [vp, vp, u32, C.POINTER(sz)]
        L.qa_integrate.argtypes = [vp, vp, vp, u64, u64, u32, u32, u32, vp, sz, vp, vp, vp]
        L.qa_allocate_budgets.argtypes = [vp, vp, u64, u64, vp]
        L.qa_autotune.argtypes = [vp, vp, vp, u64, u32, u64, vp, sz, vp, C.POINTER(u32), C.POINTER(u32),
                                  C.POINTER(C.c_double), vp]
        L.qa_variance_grad.argtypes = [vp, u32, u64, u32, u64, u64, vp, vp, vp]
        L.qa_graph_flops.argtypes = [vp, u32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.qa_dirac_trace.argtypes = [vp, i32, C.POINTER(C.c_double)]
        L.qa_results.argtypes = [vp, vp, vp, vp]
        L.qa_acc_read.argtypes = [vp, vp, vp, vp, vp]
        L.qa_combine.argtypes = [vp, sz, vp]
        L.qa_sum_results.argtypes = [vp, sz, vp]
        L.qa_pdf_with.argtypes = [vp, u32, vp, C.POINTER(vp)]
        L.qa_pdf_tune.argtypes = [vp, u32, vp, C.c_double, C.c_double, C.POINTER(vp), vp]
        L.qa_variance_gradient.argtypes = [vp, vp, u32, u64, u32, u64, u64, vp, vp, C.POINTER(C.c_double), vp]
        L.qa_acc_merge.argtypes = [vp, vp, sz]
        L.qa_pdf_create_merged.argtypes = [vp, vp, C.POINTER(vp)]
        L.qa_pdf_lines.argtypes = [vp, u32, C.POINTER(C.c_int)]
        L.qa_graph_flops_nonzero.argtypes = [vp, u32, C.POINTER(C.c_double)]
        L.qa_integrate_noalloc.argtypes = [vp, vp, vp, u64, u64, u32, u32, u32, vp, vp]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        msg = lib().qa_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed ({rc}): {msg}")


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------- graphs

def enumerate_graphs(loops, k=-1, m=-1, n=-1):
    """Canonical representatives (numpy structured array of qa_graph)."""
    cnt = C.c_size_t()
    rc = lib().qa_enumerate_graphs(loops, k, m, n, None, 0, C.byref(cnt))
    if rc not in (0, -2):
        _check(rc, "qa_enumerate_graphs")
    arr = (QaGraph * max(1, cnt.value))()
    _check(lib().qa_enumerate_graphs(loops, k, m, n, arr, cnt.value, C.byref(cnt)), "qa_enumerate_graphs")
    return list(arr)[:cnt.value]


def graph_dict(g):
    n = g.loops
    return {"n": n, "x": g.x, "mate": list(g.mate[:2 * n + 1]), "mult": g.mult, "cls": tuple(g.cls)}


class GraphSet:
    """qa_set handle: graphs, subgraphs, forests and coefficient tables."""

    def __init__(self, graphs, nthreads=0):
        self.graphs = list(graphs)
        arr = (QaGraph * len(self.graphs))(*self.graphs)
        h = C.c_void_p()
        _check(lib().qa_build_forests(arr, len(self.graphs), nthreads, C.byref(h)), "qa_build_forests")
        self.h = h

    def __len__(self):
        return len(self.graphs)

    def serialize(self):
        ln = C.c_size_t()
        lib().qa_forests_serialize(self.h, None, 0, C.byref(ln))
        buf = C.create_string_buffer(ln.value)
        _check(lib().qa_forests_serialize(self.h, buf, ln.value, C.byref(ln)), "qa_forests_serialize")
        return np.frombuffer(buf.raw, dtype="<i4").copy()

    def stats(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().qa_set_stats(self.h, C.byref(a), C.byref(b), C.byref(c)), "qa_set_stats")
        return {"terms": a.value, "blocks": b.value, "coefficients": c.value}

    def flops(self, g):
        """(evaluation, sampling) algorithmic FP64 flops per sample of graph g."""
        a, b = C.c_double(), C.c_double()
        _check(lib().qa_graph_flops(self.h, g, C.byref(a), C.byref(b)), "qa_graph_flops")
        return a.value, b.value

    def flops_nonzero(self, g):
        """Evaluation flops of graph g with the folds priced at their nonzero coefficients."""
        a = C.c_double()
        _check(lib().qa_graph_flops_nonzero(self.h, g, C.byref(a)), "qa_graph_flops_nonzero")
        return a.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.qa_set_destroy(self.h)
            self.h = None


def build_forests(graphs, nthreads=0):
    return GraphSet(graphs, nthreads)


class Pdf:
    """qa_pdf handle: Deg and W tables of eq. (1)."""

    def __init__(self, gset, deg=None, _handle=None):
        self.gset = gset
        if _handle is not None:
            self.h = _handle
            return
        h = C.c_void_p()
        dptr = None
        if deg is not None:
            self._deg = np.ascontiguousarray(np.concatenate([np.asarray(d, dtype=np.float64) for d in deg]))
            dptr = self._deg.ctypes.data_as(C.c_void_p)
        _check(lib().qa_pdf_create(gset.h, dptr, C.byref(h)), "qa_pdf_create")
        self.h = h

    def lines(self, g):
        """Lines sampled for graph g: 3n, or 3n - 1 for a merged pdf."""
        m = C.c_int()
        _check(lib().qa_pdf_lines(self.h, g, C.byref(m)), "qa_pdf_lines")
        return m.value

    def merged(self):
        """qa_pdf_create_merged: the 3n-2-variable form of this (unmerged) pdf."""
        h = C.c_void_p()
        _check(lib().qa_pdf_create_merged(self.gset.h, self.h, C.byref(h)), "qa_pdf_create_merged")
        return Pdf(self.gset, _handle=h)

    def tables(self, g):
        M = self.lines(g)
        D = np.zeros(1 << M)
        W = np.zeros(1 << M)
        _check(lib().qa_pdf_tables(self.h, g, D.ctypes.data_as(C.c_void_p), W.ctypes.data_as(C.c_void_p)),
               "qa_pdf_tables")
        return D, W

    def dlogw(self, g):
        M = self.lines(g)
        out = np.zeros(1 << M)
        _check(lib().qa_pdf_dlogw(self.h, g, out.ctypes.data_as(C.c_void_p)), "qa_pdf_dlogw")
        return out

    def with_graph(self, g, deg):
        """A new Pdf equal to this one except graph g's Deg table."""
        d = np.ascontiguousarray(deg, dtype=np.float64)
        if d.shape != (1 << self.lines(g),):
            raise RuntimeError("deg must hold 2^M entries")
        h = C.c_void_p()
        _check(lib().qa_pdf_with(self.h, g, d.ctypes.data_as(C.c_void_p), C.byref(h)), "qa_pdf_with")
        return Pdf(self.gset, _handle=h)

    def tune(self, g, grad, step, floor=0.5):
        """One pilot step on graph g (qa_pdf_tune): returns (new Pdf, shifts per set size)."""
        M = self.lines(g)
        gr = np.ascontiguousarray(grad, dtype=np.float64)
        if gr.shape != (1 << M,):
            raise RuntimeError("grad must hold 2^M entries")
        th = np.zeros(M)
        h = C.c_void_p()
        _check(lib().qa_pdf_tune(self.h, g, gr.ctypes.data_as(C.c_void_p), step, floor, C.byref(h),
                                 th.ctypes.data_as(C.c_void_p)), "qa_pdf_tune")
        return Pdf(self.gset, _handle=h), th

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.qa_pdf_destroy(self.h)
            self.h = None


def pdf_create(gset, deg=None):
    return Pdf(gset, deg)


class DeviceImage:
    """Device copy of the set's tables and the pdf (caller-owned torch buffer)."""

    def __init__(self, gset, pdf, device="cuda", stream=None):
        import torch
        n = C.c_size_t()
        _check(lib().qa_device_bytes(gset.h, pdf.h, C.byref(n)), "qa_device_bytes")
        self.buf = torch.empty(n.value, dtype=torch.uint8, device=device)
        self.gset, self.pdf = gset, pdf
        _check(lib().qa_upload(gset.h, pdf.h, _ptr(self.buf), n.value, _stream(stream)), "qa_upload")

    @property
    def ptr(self):
        return _ptr(self.buf)


def upload(gset, pdf, device="cuda", stream=None):
    return DeviceImage(gset, pdf, device, stream)


# --------------------------------------------------------------------------- hot path

def _lines(img, graph):
    if not 0 <= graph < len(img.gset.graphs):
        raise RuntimeError(f"graph index {graph} out of range (set has {len(img.gset.graphs)} graphs)")
    return 3 * img.gset.graphs[graph].loops


def sample_pdf(img, graph, seed, tag, first, count, want_sector=False, stream=None):
    import torch
    M = _lines(img, graph)
    dev = img.buf.device
    z = torch.empty((M, count), dtype=torch.float64, device=dev)
    logp = torch.empty(count, dtype=torch.float64, device=dev)
    sec = torch.empty((M, count), dtype=torch.uint8, device=dev) if want_sector else None
    _check(lib().qa_sample_pdf(img.ptr, graph, seed, tag, first, count, _ptr(z), _ptr(logp), _ptr(sec),
                               _stream(stream)), "qa_sample_pdf")
    return z, logp, sec


def eval_integrand(img, graph, z, mode=QA_FP64, stream=None):
    import torch
    M, count = z.shape
    if M != _lines(img, graph) or z.dtype != torch.float64 or not z.is_contiguous():
        raise RuntimeError("z must be a contiguous float64 tensor of shape (3n, count)")
    f = torch.empty(count, dtype=torch.float64, device=z.device)
    err = torch.empty(count, dtype=torch.float64, device=z.device) if mode != QA_FP64 else None
    flag = torch.empty(count, dtype=torch.uint8, device=z.device) if mode in (QA_FP64_BOUND, QA_FP64_EST) else None
    _check(lib().qa_eval_integrand(img.ptr, graph, _ptr(z), count, mode, _ptr(f), _ptr(err), _ptr(flag),
                                   _stream(stream)), "qa_eval_integrand")
    return f, err, flag


def new_acc(ngraphs, device="cuda"):
    import torch
    return torch.zeros(ngraphs * ACC_BYTES, dtype=torch.uint8, device=device)


def accumulate(f, logp, acc, index=0, stream=None):
    ptr = C.c_void_p(acc.data_ptr() + index * ACC_BYTES)
    _check(lib().qa_accumulate(_ptr(f), _ptr(logp), f.numel(), ptr, _stream(stream)), "qa_accumulate")


def read_acc(acc):
    return np.frombuffer(acc.cpu().numpy().tobytes(), dtype=ACC_DTYPE)


def results(gset, acc_np):
    """Per-graph and set results (qa_results) from host accumulator records:
    (numpy RESULT_DTYPE array of per-graph records, total record)."""
    rec = np.ascontiguousarray(acc_np, dtype=ACC_DTYPE)
    if rec.shape != (len(gset),):
        raise RuntimeError("need one accumulator record per graph")
    per = np.zeros(len(gset), dtype=RESULT_DTYPE)
    tot = np.zeros(1, dtype=RESULT_DTYPE)
    _check(lib().qa_results(gset.h, rec.ctypes.data_as(C.c_void_p), per.ctypes.data_as(C.c_void_p),
                            tot.ctypes.data_as(C.c_void_p)), "qa_results")
    return per, tot[0]


def acc_read(gset, acc, stream=None):
    """qa_acc_read: results straight from the device accumulators."""
    per = np.zeros(len(gset), dtype=RESULT_DTYPE)
    tot = np.zeros(1, dtype=RESULT_DTYPE)
    _check(lib().qa_acc_read(gset.h, _ptr(acc), per.ctypes.data_as(C.c_void_p), tot.ctypes.data_as(C.c_void_p),
                             _stream(stream)), "qa_acc_read")
    return per, tot[0]


def acc_merge(into, frm):
    """qa_acc_merge: into += frm (host accumulator records, equal length); returns into."""
    a = np.ascontiguousarray(into, dtype=ACC_DTYPE)
    b = np.ascontiguousarray(frm, dtype=ACC_DTYPE)
    if a.shape != b.shape:
        raise RuntimeError("records of different lengths")
    _check(lib().qa_acc_merge(a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), len(a)), "qa_acc_merge")
    return a


def combine(runs):
    """qa_combine: inverse-variance combination of independent result records."""
    r = np.ascontiguousarray(np.asarray(runs, dtype=RESULT_DTYPE).reshape(-1))
    out = np.zeros(1, dtype=RESULT_DTYPE)
    _check(lib().qa_combine(r.ctypes.data_as(C.c_void_p), len(r), out.ctypes.data_as(C.c_void_p)), "qa_combine")
    return out[0]


def sum_results(parts):
    """qa_sum_results: the sum of results of independent integrals."""
    r = np.ascontiguousarray(np.asarray(parts, dtype=RESULT_DTYPE).reshape(-1))
    out = np.zeros(1, dtype=RESULT_DTYPE)
    _check(lib().qa_sum_results(r.ctypes.data_as(C.c_void_p), len(r), out.ctypes.data_as(C.c_void_p)), "qa_sum_results")
    return out[0]


def estimates(gset, acc_np):
    """(value, sigma) per graph, as computed by the library (qa_results)."""
    per, _ = results(gset, acc_np)
    return [(float(r["value"]), float(r["sigma"])) for r in per]


def work_bytes(gset, budgets, tile=0):
    b = np.ascontiguousarray(budgets, dtype=np.uint64)
    n = C.c_size_t()
    _check(lib().qa_work_bytes(gset.h, b.ctypes.data_as(C.c_void_p), tile, C.byref(n)), "qa_work_bytes")
    return n.value


def integrate(gset, img, budgets, seed, tag=0, tile=0, grid=0, work=None, acc=None, first=0, timing=False,
              stream=None):
    """Batched form: persistent fused launches under a hipGraph.  Returns acc,
    or (acc, fused-kernel milliseconds) with timing=True."""
    import torch
    b = np.ascontiguousarray(budgets, dtype=np.uint64)
    dev = img.buf.device
    if work is None:
        work = torch.empty(work_bytes(gset, b, tile), dtype=torch.uint8, device=dev)
    if acc is None:
        acc = new_acc(len(gset), dev)
    ms = C.c_double(0.0)
    _check(lib().qa_integrate(gset.h, img.ptr, b.ctypes.data_as(C.c_void_p), first, seed, tag, tile, grid,
                              _ptr(work), work.numel(), _ptr(acc), C.byref(ms) if timing else None,
                              _stream(stream)), "qa_integrate")
    return (acc, ms.value) if timing else acc


def integrate_noalloc(gset, img, budgets, seed, tag=0, tile=0, grid=0, acc=None, first=0, stream=None):
    """qa_integrate_noalloc: the batched form on the library's scratch array
    (no work buffer, no allocation in the call; acc must be passed to keep the
    call itself allocation-free)."""
    b = np.ascontiguousarray(budgets, dtype=np.uint64)
    if acc is None:
        acc = new_acc(len(gset), img.buf.device)
    _check(lib().qa_integrate_noalloc(gset.h, img.ptr, b.ctypes.data_as(C.c_void_p), first, seed, tag, tile, grid,
                                      _ptr(acc), _stream(stream)), "qa_integrate_noalloc")
    return acc


def allocate_budgets(gset, pilot, total, floor=0):
    """Per-graph budgets from pilot sums (ACC_DTYPE records, e.g. read_acc of a
    pilot integrate): Neyman allocation mu sigma / sqrt(cost), floored, summing to total."""
    rec = np.ascontiguousarray(pilot, dtype=ACC_DTYPE)
    if rec.shape != (len(gset),):
        raise RuntimeError("pilot must hold one record per graph")
    out = np.zeros(len(gset), dtype=np.uint64)
    _check(lib().qa_allocate_budgets(gset.h, rec.ctypes.data_as(C.c_void_p), int(total), int(floor),
                                     out.ctypes.data_as(C.c_void_p)), "qa_allocate_budgets")
    return out


def autotune(gset, img, budgets, seed, tag=0, pilot=0, work=None, stream=None):
    """Pick the batched form's (tile, grid) by timing the fused pass on a pilot
    share of the budgets.  Returns (tile, grid, ns per sample)."""
    import torch
    b = np.ascontiguousarray(budgets, dtype=np.uint64)
    dev = img.buf.device
    if work is None:
        work = torch.empty(work_bytes(gset, b, 256), dtype=torch.uint8, device=dev)
    acc = new_acc(len(gset), dev)
    tile, grid, ns = C.c_uint32(), C.c_uint32(), C.c_double()
    _check(lib().qa_autotune(gset.h, img.ptr, b.ctypes.data_as(C.c_void_p), seed, tag, pilot, _ptr(work),
                             work.numel(), _ptr(acc), C.byref(tile), C.byref(grid), C.byref(ns), _stream(stream)),
           "qa_autotune")
    return tile.value, grid.value, ns.value


def variance_grad(img, graph, seed, tag, first, count, grad=None, w2sum=None, stream=None):
    import torch
    M = img.pdf.lines(graph)
    dev = img.buf.device
    if grad is None:
        grad = torch.zeros(1 << M, dtype=torch.float64, device=dev)
    if w2sum is None:
        w2sum = torch.zeros(1, dtype=torch.float64, device=dev)
    _check(lib().qa_variance_grad(img.ptr, graph, seed, tag, first, count, _ptr(grad), _ptr(w2sum),
                                  _stream(stream)), "qa_variance_grad")
    return grad, w2sum


def variance_gradient(pdf, img, graph, seed, tag, first, count, stream=None):
    """qa_variance_gradient: (E[w^2], d E[w^2] / d Deg(S) for all S) of one graph
    on samples first..first+count-1; pdf must be the one img was uploaded from."""
    import torch
    _lines(img, graph)
    M = pdf.lines(graph)
    work = torch.empty((1 << M) + 1, dtype=torch.float64, device=img.buf.device)
    grad = np.zeros(1 << M)
    m2 = C.c_double()
    _check(lib().qa_variance_gradient(pdf.h, img.ptr, graph, seed, tag, first, count, _ptr(work),
                                      grad.ctypes.data_as(C.c_void_p), C.byref(m2), _stream(stream)),
           "qa_variance_gradient")
    return m2.value, grad


def dirac_trace(symbols):
    arr = (C.c_int32 * len(symbols))(*symbols)
    out = C.c_double()
    _check(lib().qa_dirac_trace(arr, len(symbols), C.byref(out)), "qa_dirac_trace")
    return out.value


from .autograd import VarianceFn, variance_and_grad  # noqa: E402,F401
