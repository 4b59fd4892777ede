"""Python binding of the MI355X clip-alignment library (libclipalign.so).

Argument marshalling only: every step of the alignment path runs in the
library's HIP kernels.  PyTorch supplies device memory (CUDA tensors on the
ROCm build) and the current stream.  The binding fails loudly when the built
library is missing; there is no fallback implementation.

Names follow ``include/clipalign.h``: ``Context.clips`` wraps
``ca_clips_create``, ``Context.align_pairs`` wraps ``ca_align_pairs``,
``Context.prune`` wraps ``ca_prune`` and ``Context.cluster`` wraps
``ca_cluster``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclipalign.so")

CA_OK, CA_EINVAL, CA_ENOMEM, CA_EDEVICE, CA_EBUSY, CA_ETRUNC, CA_ESTATE, CA_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
CA_COSINE, CA_EDGE = 1, 2
PATHS = {"mixed": 0, "fp32": 1, "fp64": 2, "auto": 3, "direct": 4, "xcorr": 5, "xysep": 6}
CA_CLIPS_DEVICE_PTRS, CA_CLIPS_FP32, CA_CLIPS_FP64, CA_CLIPS_IMAGE, CA_CLIPS_NO_FP64 = 1, 2, 4, 8, 16
CA_CLIPS_CONTOURS = 32
CA_EDGES_BOX, CA_EDGES_CONTOUR = 0, 1
FLAG_RESCORED_FWD, FLAG_RESCORED_REV, FLAG_EMPTY = 1, 2, 4
FLAG_NO_MATCH_FWD, FLAG_NO_MATCH_REV, FLAG_RECHECK_FWD, FLAG_RECHECK_REV = 8, 16, 32, 64
FLAG_INVALID = 128
NOALLOC_MAX_PAIRS = 1 << 20

SYMBOLS = [
    "ca_create", "ca_destroy", "ca_last_error", "ca_get_stats", "ca_reset_stats",
    "ca_clips_create", "ca_clips_destroy", "ca_clips_count", "ca_clips_inspect", "ca_clips_image", "ca_clips_spectrum",
    "ca_clips_contours",
    "ca_align_pairs", "ca_align_pairs_noalloc", "ca_surface", "ca_prune", "ca_cluster", "ca_cluster_schedule",
    "ca_cover", "ca_cover_dense", "ca_verify_centers",
    "ca_server_create", "ca_server_destroy", "ca_server_submit", "ca_server_poll", "ca_server_wait",
    "ca_server_stats", "ca_server_run_stats", "ca_server_last_error",
    "ca_autotune_report", "ca_autotune_save", "ca_autotune_load", "ca_autotune_clear",
    "ca_graph_create", "ca_graph_launch", "ca_graph_invalid", "ca_graph_destroy",
    "ca_probe_read_bandwidth",
]


class ClipAlignError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"clipalign status {status}: {msg}")
        self.status = status


class _Config(C.Structure):
    _fields_ = [("device", C.c_int32), ("check_sample", C.c_int32), ("hbm_budget_bytes", C.c_uint64)]


class _Constraint(C.Structure):
    _fields_ = [("kind", C.c_int32), ("edges", C.c_int32), ("thr_num", C.c_int64), ("thr_den", C.c_int64)]


class _Stats(C.Structure):
    _fields_ = [("pairs_aligned", C.c_int64), ("pairs_rescored", C.c_int64), ("pairs_edge", C.c_int64),
                ("pairs_screened", C.c_int64), ("pairs_survived", C.c_int64),
                ("n_main_launch", C.c_int64), ("t_main_ms", C.c_double), ("main_alg_bytes", C.c_double),
                ("max_surface_err", C.c_double), ("tie_band_mixed", C.c_double),
                ("tie_band_fp32", C.c_double), ("tie_band_direct", C.c_double),
                ("max_peak_err_sqrt", C.c_double), ("groups_exact", C.c_int64),
                ("pairs_full_fp64", C.c_int64), ("cover_nnz", C.c_int64),
                ("members_verified", C.c_int64), ("center_violations", C.c_int64),
                ("check_pairs", C.c_int64), ("check_changed", C.c_int64), ("check_peak_err_sqrt", C.c_double),
                ("check_band_frac", C.c_double)]


_LIB = None
P = C.c_void_p


def load():
    """Load the built library (raises ImportError if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2512_13133_amd.build.build() first")
    lib = C.CDLL(LIB_PATH)
    lib.ca_create.argtypes = [C.POINTER(_Config), C.POINTER(P)]
    lib.ca_destroy.argtypes = [P]
    lib.ca_last_error.argtypes = [P]
    lib.ca_last_error.restype = C.c_char_p
    lib.ca_get_stats.argtypes = [P, C.POINTER(_Stats)]
    lib.ca_reset_stats.argtypes = [P]
    lib.ca_clips_create.argtypes = [P, P, C.c_int64, P, P, P, P, C.c_int32, C.POINTER(P)]
    lib.ca_clips_destroy.argtypes = [P]
    lib.ca_clips_count.argtypes = [P, C.POINTER(C.c_int64)]
    lib.ca_clips_inspect.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, P]
    lib.ca_clips_image.argtypes = [P, C.c_int64, P]
    lib.ca_clips_spectrum.argtypes = [P, C.c_int64, C.c_int32, P]
    lib.ca_clips_contours.argtypes = [P, C.c_int64, P, P, C.c_int64, P, P]
    lib.ca_align_pairs.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int32, C.c_int64,
                                   P, P, P, P, P, P, P]
    lib.ca_align_pairs_noalloc.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int32, C.c_int64,
                                           P, P, P, P, P, P, P]
    lib.ca_surface.argtypes = [P, P, P, C.c_int32, C.c_int64, P, P, P]
    lib.ca_prune.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int64, P, P, C.POINTER(C.c_int64)]
    lib.ca_cluster.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int32, C.c_int32, P, P,
                               C.POINTER(C.c_int64)]
    lib.ca_cluster_schedule.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int32, C.c_int32, C.c_int64,
                                        C.c_int64, P, P, C.POINTER(C.c_int64)]
    lib.ca_cover.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int32, C.c_int64, P, P, P, P, P,
                             C.POINTER(C.c_int64)]
    lib.ca_cover_dense.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int32, P]
    lib.ca_verify_centers.argtypes = [P, P, P, C.POINTER(_Constraint), P, P, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
    lib.ca_server_create.argtypes = [P, P, C.POINTER(_Constraint), C.c_int32, C.c_uint64, C.POINTER(P)]
    lib.ca_server_destroy.argtypes = [P]
    lib.ca_server_submit.argtypes = [P, C.c_int64, P, P, P, P, C.POINTER(C.c_uint64)]
    lib.ca_server_poll.argtypes = [P, C.c_uint64, P, P, P, P, C.POINTER(C.c_int32)]
    lib.ca_server_wait.argtypes = [P, C.c_uint64, C.c_int32]
    lib.ca_server_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]
    lib.ca_server_run_stats.argtypes = [P, C.POINTER(_Stats)]
    lib.ca_server_last_error.argtypes = [P]
    lib.ca_server_last_error.restype = C.c_char_p
    lib.ca_autotune_report.argtypes = [P, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)]
    lib.ca_autotune_save.argtypes = [P, C.c_char_p]
    lib.ca_autotune_load.argtypes = [P, C.c_char_p]
    lib.ca_autotune_clear.argtypes = [P]
    lib.ca_graph_create.argtypes = [P, P, P, C.POINTER(_Constraint), C.c_int64, P, P, P, P, P, P, P, C.POINTER(P)]
    lib.ca_graph_launch.argtypes = [P, P]
    lib.ca_graph_invalid.argtypes = [P, P, C.POINTER(C.c_int64)]
    lib.ca_graph_destroy.argtypes = [P]
    lib.ca_probe_read_bandwidth.argtypes = [P, P, C.c_uint64, C.c_int32, C.POINTER(C.c_double)]
    for name in SYMBOLS:
        if name not in ("ca_last_error", "ca_server_last_error"):
            getattr(lib, name).restype = C.c_int
    _LIB = lib
    return lib


def _ptr(a):
    """Raw address of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def constraint(kind, thr):
    """('cosine', (p, q)), ('edge', t_px) (bounding-box edges) or ('contour',
    t_px) (the edge track over full boundary edges) -> ca_constraint."""
    if kind == "cosine":
        p, q = thr
        return _Constraint(CA_COSINE, CA_EDGES_BOX, int(p), int(q))
    if kind == "edge":
        return _Constraint(CA_EDGE, CA_EDGES_BOX, int(thr), 1)
    if kind == "contour":
        return _Constraint(CA_EDGE, CA_EDGES_CONTOUR, int(thr), 1)
    raise ValueError(kind)


def probe_read_bandwidth(tensor, reps=10):
    """Milliseconds per plain streaming read of a CUDA tensor's bytes
    (``ca_probe_read_bandwidth``, on the current stream): a measurement aid."""
    import torch
    lib = load()
    ms = C.c_double(0.0)
    st = lib.ca_probe_read_bandwidth(torch.cuda.current_stream(tensor.device).cuda_stream, tensor.data_ptr(),
                                     tensor.numel() * tensor.element_size(), int(reps), C.byref(ms))
    if st != CA_OK:
        raise ClipAlignError(st, "read probe failed")
    return ms.value


class ClipSet:
    def __init__(self, ctx, handle, n):
        self.ctx, self.handle, self.n = ctx, handle, n

    def close(self):
        if self.handle:
            self.ctx._check(self.ctx.lib.ca_clips_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A library context on one GPU (``ca_create``)."""

    def __init__(self, device=0, hbm_budget_bytes=0, check_sample=0):
        import torch  # device memory and streams come from torch

        self.torch = torch
        self.lib = load()
        self.device = device
        h = P()
        st = self.lib.ca_create(C.byref(_Config(device, int(check_sample), hbm_budget_bytes)), C.byref(h))
        if st != CA_OK:
            raise ClipAlignError(st, self.lib.ca_last_error(None).decode())
        self.h = h
        self.dev = torch.device("cuda", device)

    def _check(self, st):
        if st != CA_OK:
            raise ClipAlignError(st, self.lib.ca_last_error(self.h).decode())

    def _stream(self):
        return self.torch.cuda.current_stream(self.dev).cuda_stream

    def close(self):
        if getattr(self, "h", None):
            self._check(self.lib.ca_destroy(self.h))
            self.h = None

    # -------------------------------------------------------------- clips
    def clips(self, cs, fp32=False, image=False, fp64=True, contours=False):
        """Build a device clip set from a ``clipgen.ClipSet`` (host arrays).

        fp32: keep FP32 spectra (the "fp32" path); image: keep the FP16 whitened
        images (the "direct" path); fp64=False: keep no FP64 spectra (128 x 128
        sets; the re-decision computes the ones it needs); contours: trace the
        polygon contours (the "contour" kind of the edge track)."""
        ptr = np.ascontiguousarray(cs.rect_ptr, dtype=np.int64)
        rects = np.ascontiguousarray(cs.rects, dtype=np.int32).reshape(-1, 4)
        rn = np.ascontiguousarray(cs.raster_n, dtype=np.int16)
        mw = np.ascontiguousarray(cs.marker_w, dtype=np.int16)
        flags = (CA_CLIPS_FP32 if fp32 else 0) | (CA_CLIPS_IMAGE if image else 0) | (0 if fp64 else CA_CLIPS_NO_FP64) | \
            (CA_CLIPS_CONTOURS if contours else 0)
        h = P()
        self._check(self.lib.ca_clips_create(self.h, self._stream(), rn.size, _ptr(ptr),
                                             _ptr(rects) if rects.size else None, _ptr(rn), _ptr(mw),
                                             flags, C.byref(h)))
        return ClipSet(self, h, rn.size)

    def inspect(self, clips, i, N):
        out = dict(bits=np.zeros(N * N // 64, np.uint64), n_pix=np.zeros(1, np.int32),
                   rowsum=np.zeros(N, np.uint16), colsum=np.zeros(N, np.uint16),
                   n_poly=np.zeros(1, np.int32), boxes=np.zeros((64, 4), np.int16),
                   zero_bins=np.zeros(1, np.int32), spec16=np.zeros((N, N // 2 + 1, 2), np.float32))
        self._check(self.lib.ca_clips_inspect(clips.handle, int(i), *[_ptr(out[k]) for k in (
            "bits", "n_pix", "rowsum", "colsum", "n_poly", "boxes", "zero_bins", "spec16")]))
        return out

    def image(self, clips, i, N):
        """Whitened image N * IDFT2(W) of clip i as stored (FP16 widened), [N, N]."""
        out = np.zeros((N, N), np.float32)
        self._check(self.lib.ca_clips_image(clips.handle, int(i), _ptr(out)))
        return out

    def spectrum(self, clips, i, N, precision=64):
        """Stored whitened half-spectrum of clip i, complex128 [N, N/2 + 1]."""
        out = np.zeros((N, N // 2 + 1, 2), np.float64)
        self._check(self.lib.ca_clips_spectrum(clips.handle, int(i), int(precision), _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def contours(self, clips, i):
        """Contour tables of clip i: dict(n_edges, edges uint16, poly_ptr
        uint16[65], hashes uint32[64]); n_edges -1 without contour data."""
        ne = C.c_int32(0)
        pp = np.zeros(65, np.uint16)
        hs = np.zeros(64, np.uint32)
        self._check(self.lib.ca_clips_contours(clips.handle, int(i), C.byref(ne), None, 0, _ptr(pp), _ptr(hs)))
        edges = np.zeros(max(ne.value, 0), np.uint16)
        if ne.value > 0:
            self._check(self.lib.ca_clips_contours(clips.handle, int(i), None, _ptr(edges), edges.size, None, None))
        return dict(n_edges=ne.value, edges=edges, poly_ptr=pp, hashes=hs)

    # -------------------------------------------------------------- pairs
    def align_pairs(self, clips, rep, mem, kind="cosine", thr=(19, 20), path="mixed", noalloc=False):
        """Align unordered pairs on the GPU; returns a dict of CUDA tensors.
        noalloc=True calls ca_align_pairs_noalloc (no device allocation inside
        the library; at most NOALLOC_MAX_PAIRS pairs)."""
        torch = self.torch
        rep = torch.as_tensor(rep, dtype=torch.int32, device=self.dev).contiguous()
        mem = torch.as_tensor(mem, dtype=torch.int32, device=self.dev).contiguous()
        n = rep.numel()
        out = dict(
            bits=torch.empty(n, dtype=torch.uint8, device=self.dev),
            shift=torch.empty((n, 2, 2), dtype=torch.int16, device=self.dev),
            count=torch.empty((n, 2), dtype=torch.int32, device=self.dev),
            score=torch.empty((n, 2), dtype=torch.float64, device=self.dev),
            flags=torch.empty(n, dtype=torch.int32, device=self.dev),
        )
        con = constraint(kind, thr)
        fn = self.lib.ca_align_pairs_noalloc if noalloc else self.lib.ca_align_pairs
        self._check(fn(self.h, self._stream(), clips.handle, C.byref(con), PATHS[path], n, _ptr(rep), _ptr(mem),
                       _ptr(out["bits"]), _ptr(out["shift"]), _ptr(out["count"]), _ptr(out["score"]),
                       _ptr(out["flags"])))
        return out

    def surface(self, clips, rep, mem, path="mixed"):
        """Low-precision window surfaces [n, 33, 33] (direction 0), normalised by K_hi."""
        torch = self.torch
        rep = torch.as_tensor(rep, dtype=torch.int32, device=self.dev).contiguous()
        mem = torch.as_tensor(mem, dtype=torch.int32, device=self.dev).contiguous()
        surf = torch.zeros((rep.numel(), 33, 33), dtype=torch.float32, device=self.dev)
        self._check(self.lib.ca_surface(self.h, self._stream(), clips.handle, PATHS[path], rep.numel(),
                                        _ptr(rep), _ptr(mem), _ptr(surf)))
        return surf

    def prune(self, clips, kind="cosine", thr=(19, 20)):
        """Candidate pairs surviving the safe bounds: (rep, mem) CUDA int32 tensors."""
        torch = self.torch
        con = constraint(kind, thr)
        n = C.c_int64(0)
        self._check(self.lib.ca_prune(self.h, self._stream(), clips.handle, C.byref(con), 0, None, None,
                                      C.byref(n)))
        rep = torch.empty(max(n.value, 1), dtype=torch.int32, device=self.dev)
        mem = torch.empty(max(n.value, 1), dtype=torch.int32, device=self.dev)
        got = C.c_int64(0)
        if n.value:
            self._check(self.lib.ca_prune(self.h, self._stream(), clips.handle, C.byref(con), n.value,
                                          _ptr(rep), _ptr(mem), C.byref(got)))
        return rep[:n.value], mem[:n.value]

    def cluster(self, clips, kind="cosine", thr=(19, 20), iterations=1, path="mixed", relax=None):
        """Full method; returns dict(rep_of, center_shift, n_clusters) as numpy.
        ``relax``: the schedule's relaxation ((num, den) for the cosine track,
        pixels per step for the edge track; ``ca_cluster_schedule``), or None
        for the default."""
        rep_of = np.zeros(clips.n, np.int32)
        shift = np.zeros((clips.n, 2), np.int16)
        k = C.c_int64(0)
        con = constraint(kind, thr)
        if relax is None:
            self._check(self.lib.ca_cluster(self.h, self._stream(), clips.handle, C.byref(con), PATHS[path],
                                            int(iterations), _ptr(rep_of), _ptr(shift), C.byref(k)))
        else:
            rn, rd = relax if isinstance(relax, tuple) else (int(relax), 1)
            self._check(self.lib.ca_cluster_schedule(self.h, self._stream(), clips.handle, C.byref(con), PATHS[path],
                                                     int(iterations), int(rn), int(rd), _ptr(rep_of), _ptr(shift),
                                                     C.byref(k)))
        return dict(rep_of=rep_of, center_shift=shift, n_clusters=int(k.value))

    def cover(self, clips, kind="cosine", thr=(19, 20), path="mixed"):
        """The cover relation as a CSR (``ca_cover``): dict(row_ptr, col, shift,
        value, score) of CUDA tensors, rows sorted by member."""
        torch = self.torch
        con = constraint(kind, thr)
        z = C.c_int64(0)
        self._check(self.lib.ca_cover(self.h, self._stream(), clips.handle, C.byref(con), PATHS[path], 0,
                                      None, None, None, None, None, C.byref(z)))
        nnz = z.value
        m = max(nnz, 1)
        out = dict(row_ptr=torch.empty(clips.n + 1, dtype=torch.int64, device=self.dev),
                   col=torch.empty(m, dtype=torch.int32, device=self.dev),
                   shift=torch.empty((m, 2), dtype=torch.int16, device=self.dev),
                   value=torch.empty(m, dtype=torch.int32, device=self.dev),
                   score=torch.empty(m, dtype=torch.float64, device=self.dev))
        self._check(self.lib.ca_cover(self.h, self._stream(), clips.handle, C.byref(con), PATHS[path], nnz,
                                      _ptr(out["row_ptr"]), _ptr(out["col"]), _ptr(out["shift"]),
                                      _ptr(out["value"]), _ptr(out["score"]), C.byref(z)))
        for k in ("col", "shift", "value", "score"):
            out[k] = out[k][:nnz]
        return out

    def cover_dense(self, clips, kind="cosine", thr=(19, 20), path="mixed"):
        """Dense cover bits (``ca_cover_dense``) as a uint64 CUDA tensor [n, ceil(n/64)]."""
        torch = self.torch
        con = constraint(kind, thr)
        words = (clips.n + 63) // 64
        out = torch.empty((clips.n, words), dtype=torch.int64, device=self.dev)
        self._check(self.lib.ca_cover_dense(self.h, self._stream(), clips.handle, C.byref(con), PATHS[path],
                                            _ptr(out)))
        return out

    def verify_centers(self, clips, rep_of, center_shift, kind="cosine", thr=(19, 20)):
        """(violations, first violating clip or -1) of an assignment (``ca_verify_centers``)."""
        rep_of = np.ascontiguousarray(rep_of, dtype=np.int32)
        center_shift = np.ascontiguousarray(center_shift, dtype=np.int16).reshape(-1, 2)
        con = constraint(kind, thr)
        v, f = C.c_int64(0), C.c_int64(0)
        self._check(self.lib.ca_verify_centers(self.h, self._stream(), clips.handle, C.byref(con), _ptr(rep_of),
                                               _ptr(center_shift), C.byref(v), C.byref(f)))
        return int(v.value), int(f.value)

    def graph(self, clips, n_pairs, thr=(19, 20)):
        """A captured CA_PATH_MIXED cosine alignment of a fixed pair buffer (``ca_graph_*``)."""
        return Graph(self, clips, n_pairs, thr)

    def autotune_report(self):
        """Tuned buckets of CA_PATH_AUTO, one text line each."""
        n = C.c_int64(0)
        self._check(self.lib.ca_autotune_report(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value + 1)
        self._check(self.lib.ca_autotune_report(self.h, buf, n.value + 1, C.byref(n)))
        return buf.value.decode()

    def autotune_save(self, path):
        self._check(self.lib.ca_autotune_save(self.h, str(path).encode()))

    def autotune_load(self, path):
        self._check(self.lib.ca_autotune_load(self.h, str(path).encode()))

    def autotune_clear(self):
        self._check(self.lib.ca_autotune_clear(self.h))

    def stats(self):
        s = _Stats()
        self._check(self.lib.ca_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def reset_stats(self):
        self._check(self.lib.ca_reset_stats(self.h))


class Graph:
    """Replayable alignment of ``n_pairs`` pairs: write ids with ``set_pairs``,
    then ``launch``; results live in ``out`` (CUDA tensors)."""

    def __init__(self, ctx, clips, n_pairs, thr=(19, 20)):
        torch = ctx.torch
        self.ctx, self.lib, self.clips, self.n = ctx, ctx.lib, clips, int(n_pairs)
        self.rep = torch.zeros(self.n, dtype=torch.int32, device=ctx.dev)
        self.mem = torch.zeros(self.n, dtype=torch.int32, device=ctx.dev)
        self.out = dict(
            bits=torch.empty(self.n, dtype=torch.uint8, device=ctx.dev),
            shift=torch.empty((self.n, 2, 2), dtype=torch.int16, device=ctx.dev),
            count=torch.empty((self.n, 2), dtype=torch.int32, device=ctx.dev),
            score=torch.empty((self.n, 2), dtype=torch.float64, device=ctx.dev),
            flags=torch.empty(self.n, dtype=torch.int32, device=ctx.dev),
        )
        con = constraint("cosine", thr)
        self.h = P()
        ctx._check(self.lib.ca_graph_create(ctx.h, ctx._stream(), clips.handle, C.byref(con), self.n,
                                            _ptr(self.rep), _ptr(self.mem), _ptr(self.out["bits"]),
                                            _ptr(self.out["shift"]), _ptr(self.out["count"]),
                                            _ptr(self.out["score"]), _ptr(self.out["flags"]), C.byref(self.h)))

    def set_pairs(self, rep, mem):
        torch = self.ctx.torch
        self.rep.copy_(torch.as_tensor(rep, dtype=torch.int32))
        self.mem.copy_(torch.as_tensor(mem, dtype=torch.int32))

    def launch(self):
        self.ctx._check(self.lib.ca_graph_launch(self.h, self.ctx._stream()))

    def invalid(self):
        n = C.c_int64(0)
        self.ctx._check(self.lib.ca_graph_invalid(self.h, self.ctx._stream(), C.byref(n)))
        return int(n.value)

    def close(self):
        if self.h:
            self.lib.ca_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching matcher against a device-resident library (``ca_server_*``)."""

    def __init__(self, ctx, library, thr=(19, 20), slots=4, hbm_budget_bytes=0):
        self.ctx, self.lib = ctx, ctx.lib
        self.library = library  # keep the library clip set alive
        h = P()
        con = constraint("cosine", thr)
        ctx._check(self.lib.ca_server_create(ctx.h, library.handle, C.byref(con), int(slots),
                                             int(hbm_budget_bytes), C.byref(h)))
        self.h = h

    def _check(self, st):
        if st != CA_OK:
            raise ClipAlignError(st, self.lib.ca_server_last_error(self.h).decode())

    def submit(self, cs):
        """Submit a ``clipgen.ClipSet`` batch; returns the request id (raises on refusal)."""
        ptr = np.ascontiguousarray(cs.rect_ptr, dtype=np.int64)
        rects = np.ascontiguousarray(cs.rects, dtype=np.int32).reshape(-1, 4)
        rn = np.ascontiguousarray(cs.raster_n, dtype=np.int16)
        mw = np.ascontiguousarray(cs.marker_w, dtype=np.int16)
        rid = C.c_uint64(0)
        self._check(self.lib.ca_server_submit(self.h, rn.size, _ptr(ptr), _ptr(rects) if rects.size else None,
                                              _ptr(rn), _ptr(mw), C.byref(rid)))
        return rid.value

    def poll(self, rid, n):
        """None while running, else dict(best_rep, shift, score, matched) as numpy arrays."""
        out = dict(best_rep=np.zeros(n, np.int32), shift=np.zeros((n, 2), np.int16),
                   score=np.zeros(n, np.float64), matched=np.zeros(n, np.uint8))
        done = C.c_int32(0)
        self._check(self.lib.ca_server_poll(self.h, C.c_uint64(rid), _ptr(out["best_rep"]), _ptr(out["shift"]),
                                            _ptr(out["score"]), _ptr(out["matched"]), C.byref(done)))
        return out if done.value else None

    def wait(self, rid, timeout_ms=-1):
        self._check(self.lib.ca_server_wait(self.h, C.c_uint64(rid), int(timeout_ms)))

    def run_stats(self):
        """Summed run statistics of the slots (``ca_server_run_stats``)."""
        s = _Stats()
        self._check(self.lib.ca_server_run_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def stats(self):
        a, b, c = C.c_int64(0), C.c_int64(0), C.c_uint64(0)
        self._check(self.lib.ca_server_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(requests_done=a.value, candidate_pairs=b.value, inflight_bytes=c.value)

    def close(self):
        if getattr(self, "h", None):
            self._check(self.lib.ca_server_destroy(self.h))
            self.h = None
