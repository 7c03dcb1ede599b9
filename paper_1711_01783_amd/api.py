"""Python-level API: code handles, syndrome and decode (argument marshalling)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from ._lib import (MET_BATCH_JOB_STREAMS, MET_BATCH_JOBS_IN_TURN, MET_BATCH_KIND_STREAMS, MET_BATCH_NO_GRAPH, MET_BATCH_NO_STAGGER,
                   MET_BATCH_PHASE_LAUNCHES, MET_C2V_FP16, MET_C2V_Q8, MET_CHECK_LUT, MET_FIXED_ITERS, MET_NO_COMPACT, MET_NO_DEG1_SKIP, check, lib,
                   met_check_class,
                   met_code_stats, met_job, met_kernel_time, met_profile, met_tuning)


class Code:
    """An owned ``met_code`` handle."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        st = met_code_stats()
        check(lib.met_code_info(self._h, ctypes.byref(st)))
        self.N = int(st.N)
        self.M = int(st.M)
        self.E = int(st.E)
        self._stats = st

    @staticmethod
    def _profile(profile):
        t = len(profile.vn_types[0][1])
        vfrac = (ctypes.c_double * len(profile.vn_types))(*[f for f, _ in profile.vn_types])
        vdeg = (ctypes.c_int32 * (len(profile.vn_types) * t))(*[d for _, ds in profile.vn_types for d in ds])
        cfrac = (ctypes.c_double * len(profile.cn_types))(*[f for f, _ in profile.cn_types])
        cdeg = (ctypes.c_int32 * (len(profile.cn_types) * t))(*[d for _, ds in profile.cn_types for d in ds])
        # the arrays travel with the struct so that they outlive the call
        return met_profile(t, len(profile.vn_types), vfrac, vdeg, len(profile.cn_types), cfrac, cdeg), \
            (vfrac, vdeg, cfrac, cdeg)

    @classmethod
    def build(cls, profile, n: int, seed: int) -> "Code":
        """From a degree profile with ``vn_types`` / ``cn_types`` rows of
        (fraction, per-edge-type degrees): seeded random socket permutation."""
        p, _keep = cls._profile(profile)
        h = ctypes.c_void_p()
        check(lib.met_code_build(ctypes.byref(p), int(n), int(seed) & (2**64 - 1), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def build_peg(cls, profile, n: int, seed: int, depth=None) -> "Code":
        """Progressive edge growth (met_code_build_peg); depth: search depth
        per edge type, or None for the library's default."""
        p, _keep = cls._profile(profile)
        dep = None
        if depth is not None:
            dep = (ctypes.c_int32 * len(depth))(*[int(x) for x in depth])
        h = ctypes.c_void_p()
        check(lib.met_code_build_peg(ctypes.byref(p), int(n), int(seed) & (2**64 - 1), dep, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def from_edges(cls, n: int, m: int, vn, cn, etype=None) -> "Code":
        vn = np.ascontiguousarray(vn, dtype=np.int32)
        cn = np.ascontiguousarray(cn, dtype=np.int32)
        et = None if etype is None else np.ascontiguousarray(etype, dtype=np.int8)
        h = ctypes.c_void_p()
        check(
            lib.met_code_from_edges(
                int(n), int(m), int(vn.size), vn.ctypes.data, cn.ctypes.data,
                None if et is None else et.ctypes.data, ctypes.byref(h),
            )
        )
        return cls(h)

    def info(self) -> dict:
        st = self._stats
        return {
            "N": int(st.N),
            "M": int(st.M),
            "E": int(st.E),
            "E_type": [int(st.E_type[k]) for k in range(int(st.n_edge_types))],
            "n_deg1": int(st.n_deg1),
            "edges_to_pass": int(st.edges_to_pass),
            "n_msg_vn": int(st.n_msg_vn),
            "n_msg_edges": int(st.n_msg_edges),
            "n_leaf_edges": int(st.n_leaf_edges),
            "n_edge_types": int(st.n_edge_types),
            "n_check_classes": int(st.n_check_classes),
            "max_check_degree": int(st.max_check_degree),
            "max_vn_degree": int(st.max_vn_degree),
        }

    def classes(self) -> list:
        """Check classes: dicts with n_msg, n_leaf (-1 for mixed runs),
        first_check, n_checks, n_msg_vn_touched."""
        buf = (met_check_class * 64)()
        n = ctypes.c_int32()
        check(lib.met_code_classes(self._h, buf, 64, ctypes.byref(n)))
        return [
            {f: int(getattr(buf[k], f)) for f, _ in met_check_class._fields_} for k in range(min(64, n.value))
        ]

    def export(self):
        """(vn int32 [E], cn int32 [E], etype int8 [E]) in check order."""
        vn = np.empty(self.E, dtype=np.int32)
        cn = np.empty(self.E, dtype=np.int32)
        et = np.empty(self.E, dtype=np.int8)
        check(lib.met_code_export(self._h, vn.ctypes.data, cn.ctypes.data, et.ctypes.data))
        return vn, cn, et

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib.met_code_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require(t, dtype, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def syndrome(code: Code, bits, stream=None):
    """H x mod 2 on the GPU: bits uint8 [B, N] -> uint8 [B, M]."""
    import torch

    b = int(bits.shape[0])
    _require(bits, torch.uint8, (b, code.N), "bits")
    out = torch.empty((b, code.M), dtype=torch.uint8, device=bits.device)
    check(lib.met_syndrome(code.handle, bits.data_ptr(), b, out.data_ptr(), _stream_ptr(stream)))
    return out


def mdr_bob(y, bits, d: int = 8, stream=None):
    """Bob's side of multidimensional reconciliation: (alpha float32 [B, N],
    |y| float32 [B, N/d]) from his Gaussian variables y float32 [B, N] and his
    random bits uint8 [B, N] (met_mdr_bob)."""
    import torch

    b, n = int(y.shape[0]), int(y.shape[1])
    _require(y, torch.float32, (b, n), "y")
    _require(bits, torch.uint8, (b, n), "bits")
    alpha = torch.empty((b, n), dtype=torch.float32, device=y.device)
    ynorm = torch.empty((b, max(n // d, 1)), dtype=torch.float32, device=y.device)
    check(lib.met_mdr_bob(y.data_ptr(), bits.data_ptr(), b, n, int(d), alpha.data_ptr(), ynorm.data_ptr(),
                          _stream_ptr(stream)))
    return alpha, ynorm


def mdr_alice(x, alpha, ynorm, sigma_z2: float, d: int = 8, stream=None):
    """Alice's side: decoder LLRs float32 [B, N] from her variables x, Bob's
    alpha and |y|, and the noise variance of y - x (met_mdr_alice)."""
    import torch

    b, n = int(x.shape[0]), int(x.shape[1])
    _require(x, torch.float32, (b, n), "x")
    _require(alpha, torch.float32, (b, n), "alpha")
    _require(ynorm, torch.float32, (b, max(n // d, 1)), "ynorm")
    llr = torch.empty((b, n), dtype=torch.float32, device=x.device)
    check(lib.met_mdr_alice(x.data_ptr(), alpha.data_ptr(), ynorm.data_ptr(), float(sigma_z2), b, n, int(d),
                            llr.data_ptr(), _stream_ptr(stream)))
    return llr


def workspace_bytes(code: Code, frames: int, fixed_iters: bool = False, posterior: bool = False,
                    deg1_skip: bool = True, c2v_fp16: bool = False, c2v_q8: bool = False) -> int:
    n = ctypes.c_size_t()
    flags = ((MET_FIXED_ITERS if fixed_iters else 0) | (0 if deg1_skip else MET_NO_DEG1_SKIP)
             | (MET_C2V_FP16 if c2v_fp16 else 0) | (MET_C2V_Q8 if c2v_q8 else 0))
    check(lib.met_decode_workspace_bytes(code.handle, int(frames), flags, int(bool(posterior)), ctypes.byref(n)))
    return int(n.value)


@dataclass
class DecodeOutput:
    bits: "object"       # uint8 [B, N]
    iterations: "object" # int32 [B]
    converged: "object"  # uint8 [B]
    posterior: "object"  # float32 [B, N] or None


def decode(code: Code, llr, syn, max_iter: int, fixed_iters: bool = False, posterior: bool = False,
           workspace=None, stream=None, check_steps_per_wave: int = 0, variable_chunk: int = 0,
           compact: bool = True, deg1_skip: bool = True, c2v_fp16: bool = False,
           c2v_q8: bool = False, check_lut: bool = False) -> DecodeOutput:
    """Decode llr float32 [B, N] against syn uint8 [B, M] (device tensors).

    check_steps_per_wave and variable_chunk (0 = default) select launch shapes
    of the check and variable kernels, compact=False keeps running frames in
    their groups; results do not depend on any of them.  deg1_skip=False
    iterates degree-1 variable nodes like the others (MET_NO_DEG1_SKIP; equal
    results up to FP32 rounding).  c2v_fp16=True stores check-to-variable
    messages in half precision (MET_C2V_FP16; more than 32 frames), c2v_q8=True
    in 8 bits (MET_C2V_Q8; more than 32 frames); check_lut=True (with c2v_q8)
    runs the table-driven check update (MET_CHECK_LUT)."""
    import torch

    b = int(llr.shape[0])
    dev = llr.device
    _require(llr, torch.float32, (b, code.N), "llr")
    _require(syn, torch.uint8, (b, code.M), "syn")
    need = workspace_bytes(code, b, fixed_iters, posterior, deg1_skip, c2v_fp16, c2v_q8)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-workspace.data_ptr()) % 256
    ws_ptr = workspace.data_ptr() + off
    ws_len = workspace.numel() - off
    bits = torch.empty((b, code.N), dtype=torch.uint8, device=dev)
    iters = torch.empty(b, dtype=torch.int32, device=dev)
    conv = torch.empty(b, dtype=torch.uint8, device=dev)
    post = torch.empty((b, code.N), dtype=torch.float32, device=dev) if posterior else None
    tuning = met_tuning()
    tuning.check_steps_per_wave = int(check_steps_per_wave)
    tuning.variable_chunk = int(variable_chunk)
    check(
        lib.met_decode_ex(
            code.handle, llr.data_ptr(), syn.data_ptr(), b, int(max_iter),
            (MET_FIXED_ITERS if fixed_iters else 0) | (0 if compact else MET_NO_COMPACT)
            | (0 if deg1_skip else MET_NO_DEG1_SKIP) | (MET_C2V_FP16 if c2v_fp16 else 0)
            | (MET_C2V_Q8 if c2v_q8 else 0) | (MET_CHECK_LUT if check_lut else 0),
            bits.data_ptr(), iters.data_ptr(), conv.data_ptr(),
            None if post is None else post.data_ptr(),
            ctypes.c_void_p(ws_ptr), ws_len, ctypes.byref(tuning), _stream_ptr(stream),
        )
    )
    return DecodeOutput(bits, iters, conv, post)


def decode_noalloc(code: Code, llr, syn, max_iter: int, bits, iterations, converged, posterior=None,
                   fixed_iters: bool = False, stream=None) -> None:
    """met_decode_noalloc: decode into caller-provided outputs (bits uint8
    [B, N], iterations int32 [B], converged uint8 [B], posterior float32 [B, N]
    or None) with the library's fixed device workspace; nothing is allocated
    here or in the library.  The code must already be on the device (any
    decode or syndrome call there uploads it)."""
    import torch

    b = int(llr.shape[0])
    _require(llr, torch.float32, (b, code.N), "llr")
    _require(syn, torch.uint8, (b, code.M), "syn")
    _require(bits, torch.uint8, (b, code.N), "bits")
    _require(iterations, torch.int32, (b,), "iterations")
    _require(converged, torch.uint8, (b,), "converged")
    if posterior is not None:
        _require(posterior, torch.float32, (b, code.N), "posterior")
    check(
        lib.met_decode_noalloc(
            code.handle, llr.data_ptr(), syn.data_ptr(), b, int(max_iter), MET_FIXED_ITERS if fixed_iters else 0,
            bits.data_ptr(), iterations.data_ptr(), converged.data_ptr(),
            None if posterior is None else posterior.data_ptr(), _stream_ptr(stream),
        )
    )


@dataclass
class Job:
    """One decode job of a batched call: a code, its frames and a budget."""
    code: Code
    llr: "object"        # float32 [B, N] device tensor
    syn: "object"        # uint8 [B, M] device tensor
    max_iter: int
    fixed_iters: bool = False


def _job_structs(jobs, outs):
    arr = (met_job * len(jobs))()
    for k, (j, o) in enumerate(zip(jobs, outs)):
        b = int(j.llr.shape[0])
        arr[k].code = j.code.handle
        arr[k].llr = j.llr.data_ptr()
        arr[k].syn = j.syn.data_ptr()
        arr[k].B = b
        arr[k].max_iter = int(j.max_iter)
        arr[k].flags = MET_FIXED_ITERS if j.fixed_iters else 0
        if o is not None:
            arr[k].bits = o.bits.data_ptr()
            arr[k].iters = o.iterations.data_ptr()
            arr[k].converged = o.converged.data_ptr()
        else:  # sizing only: any non-NULL aligned value passes validation
            arr[k].bits = arr[k].iters = arr[k].converged = 256
        arr[k].posterior = None
    return arr


def batched_workspace_bytes(jobs) -> int:
    arr = _job_structs(jobs, [None] * len(jobs))
    n = ctypes.c_size_t()
    check(lib.met_batched_workspace_bytes(arr, len(jobs), ctypes.byref(n)))
    return int(n.value)


class BatchedDecoder:
    """Decodes a list of jobs in one HIP graph (met_decode_batched): one
    persistent launch, or one launch per phase (phase_launches=True).

    Keeps its workspace between calls, so repeated calls with the same jobs
    replay the same cached HIP graph.  check_steps_per_wave / blocks_per_cu /
    stagger / graph / interleave (frames per group: 16, 32 or 64) /
    phase_launches / streams select launch shapes; results do not depend on
    them.  streams (phase launches only): "one" (default), "kinds" (the
    launches of a phase on parallel streams), "jobs" (each job's launches a
    chain of their own on parallel streams) or "serial" (those chains one job
    after the other)."""

    _STREAMS = {"one": 0, "kinds": MET_BATCH_KIND_STREAMS, "jobs": MET_BATCH_JOB_STREAMS,
                "serial": MET_BATCH_JOBS_IN_TURN}

    def __init__(self, check_steps_per_wave: int = 0, blocks_per_cu: int = 0, stagger: bool = True,
                 graph: bool = True, interleave: int = 0, phase_launches: bool = False, streams: str = "one"):
        if streams not in self._STREAMS:
            raise ValueError("streams must be one of %s" % sorted(self._STREAMS))
        self.tuning = met_tuning()
        self.tuning.check_steps_per_wave = int(check_steps_per_wave)
        self.tuning.blocks_per_cu = int(blocks_per_cu)
        self.tuning.interleave = int(interleave)
        self.tuning.batch_flags = ((0 if stagger else MET_BATCH_NO_STAGGER) | (0 if graph else MET_BATCH_NO_GRAPH)
                                   | (MET_BATCH_PHASE_LAUNCHES if phase_launches else 0) | self._STREAMS[streams])
        self.workspace = None
        self._ws_ptr = 0

    def __call__(self, jobs, outputs=None, stream=None):
        import torch

        if not jobs:
            raise ValueError("no jobs")
        dev = jobs[0].llr.device
        for j in jobs:
            b = int(j.llr.shape[0])
            _require(j.llr, torch.float32, (b, j.code.N), "llr")
            _require(j.syn, torch.uint8, (b, j.code.M), "syn")
        if outputs is None:
            outputs = []
            for j in jobs:
                b = int(j.llr.shape[0])
                outputs.append(DecodeOutput(torch.empty((b, j.code.N), dtype=torch.uint8, device=dev),
                                            torch.empty(b, dtype=torch.int32, device=dev),
                                            torch.empty(b, dtype=torch.uint8, device=dev), None))
        self._ensure_workspace(jobs)
        arr = _job_structs(jobs, outputs)
        ws_len = self.workspace.numel() - (self._ws_ptr - self.workspace.data_ptr())
        check(lib.met_decode_batched(arr, len(jobs), ctypes.c_void_p(self._ws_ptr), ws_len,
                                     ctypes.byref(self.tuning), _stream_ptr(stream)))
        return outputs

    def _ensure_workspace(self, jobs):
        import torch

        need = batched_workspace_bytes(jobs)
        if self.workspace is None or self.workspace.numel() - 256 < need:
            self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=jobs[0].llr.device)
            self._ws_ptr = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256

    def autotune(self, jobs, probe_iters: int = 0, stream=None) -> dict:
        """Picks this decoder's launch shape for `jobs` with the library's
        autotuner (short timed runs of the same jobs; cached per process).
        Overwrites nothing but scratch outputs; returns the chosen shape."""
        import torch

        dev = jobs[0].llr.device
        outs = [DecodeOutput(torch.empty((int(j.llr.shape[0]), j.code.N), dtype=torch.uint8, device=dev),
                             torch.empty(int(j.llr.shape[0]), dtype=torch.int32, device=dev),
                             torch.empty(int(j.llr.shape[0]), dtype=torch.uint8, device=dev), None) for j in jobs]
        self._ensure_workspace(jobs)
        arr = _job_structs(jobs, outs)
        best = met_tuning()
        ms = ctypes.c_float()
        ws_len = self.workspace.numel() - (self._ws_ptr - self.workspace.data_ptr())
        check(lib.met_batched_autotune(arr, len(jobs), ctypes.c_void_p(self._ws_ptr), ws_len, int(probe_iters),
                                       ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)))
        graph = not (self.tuning.batch_flags & MET_BATCH_NO_GRAPH)
        self.tuning = best
        keep = (MET_BATCH_NO_STAGGER | MET_BATCH_PHASE_LAUNCHES | MET_BATCH_KIND_STREAMS | MET_BATCH_JOB_STREAMS
                | MET_BATCH_JOBS_IN_TURN)
        self.tuning.batch_flags = (best.batch_flags & keep) | (0 if graph else MET_BATCH_NO_GRAPH)
        return {"schedule": "phase launches" if best.batch_flags & MET_BATCH_PHASE_LAUNCHES else "persistent",
                "streams": ("kinds" if best.batch_flags & MET_BATCH_KIND_STREAMS else
                            "jobs" if best.batch_flags & MET_BATCH_JOB_STREAMS else
                            "serial" if best.batch_flags & MET_BATCH_JOBS_IN_TURN else "one"),
                "check_steps_per_wave": int(best.check_steps_per_wave), "blocks_per_cu": int(best.blocks_per_cu),
                "interleave": int(best.interleave),
                "stagger": not (best.batch_flags & MET_BATCH_NO_STAGGER), "probe_ms": float(ms.value)}

    def barrier_expired(self) -> bool:
        """True if the last launch's grid barrier timed out (results invalid).
        Synchronises with the device."""
        e = ctypes.c_int32()
        check(lib.met_batched_check(ctypes.c_void_p(self._ws_ptr), ctypes.byref(e)))
        return bool(e.value)


def decode_batched(jobs, stream=None, **tuning):
    """One-shot batched decode; returns a DecodeOutput per job."""
    return BatchedDecoder(**tuning)(jobs, stream=stream)


def timing_enable(on: bool = True) -> None:
    """Bracket every decoder kernel launch with HIP events on its stream."""
    check(lib.met_timing_enable(1 if on else 0))


def timing_collect() -> dict:
    """{kernel name: (launches, total milliseconds)} since the last collect."""
    buf = (met_kernel_time * 64)()
    n = ctypes.c_int32()
    check(lib.met_timing_collect(buf, 64, ctypes.byref(n)))
    return {buf[k].name.decode(): (int(buf[k].launches), float(buf[k].total_ms)) for k in range(n.value)}
