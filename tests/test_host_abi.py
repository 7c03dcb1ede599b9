"""Host-side tests of the C ABI (no GPU): construction parity, validation, exports."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1711_01783_amd as met
from paper_1711_01783_amd import _lib
from oracle import code as oc
from met_inputs import PROFILES, Profile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "met_bp.h")).read()
    names = set(re.findall(r"\b(met_[a-z_0-9]+)\s*\(", hdr))
    assert {"met_code_build", "met_decode", "met_syndrome", "met_last_error"} <= names
    so = ctypes.CDLL(_lib.library_path)
    for n in sorted(names):
        assert hasattr(so, n), n


@pytest.mark.parametrize("name", list(PROFILES))
@pytest.mark.parametrize("n,seed", [(4096, 1), (20000, 7), (65536, 123456789)])
def test_cpp_builder_matches_oracle_construction(name, n, seed):
    prof = PROFILES[name]
    a = oc.build(prof, n, seed)
    b = met.Code.build(prof, n, seed)
    vn, cn, et = b.export()
    assert b.N == a.n and b.M == a.m and b.E == a.e
    np.testing.assert_array_equal(vn, a.v)
    np.testing.assert_array_equal(cn, a.c)
    np.testing.assert_array_equal(et, a.t)
    st = b.info()
    sa = a.stats()
    for k in ("N", "M", "E", "E_type", "n_deg1", "edges_to_pass"):
        assert st[k] == sa[k], k


def test_cpp_builder_repairs_like_oracle():
    prof = Profile("dense", 0.5, vn_types=((1.0, (3,)),), cn_types=((0.5, (6,)),))
    for seed in range(5):
        a = oc.build(prof, 40, seed)
        vn, cn, et = met.Code.build(prof, 40, seed).export()
        np.testing.assert_array_equal(vn, a.v)
        np.testing.assert_array_equal(cn, a.c)


def test_full_length_statistics():
    """Rate-0.1 profile at N = 10^6 (Table 1 style bookkeeping)."""
    st = met.Code.build(PROFILES["r0.1"], 10**6, 2024).info()
    assert (st["M"], st["E"], st["n_deg1"], st["edges_to_pass"]) == (900000, 3760000, 880000, 2880000)
    assert st["n_msg_vn"] == 120000 and st["n_msg_edges"] == 2880000 and st["n_leaf_edges"] == 880000
    assert st["max_check_degree"] == 12 and st["max_vn_degree"] == 24
    assert st["n_check_classes"] == 2


def test_check_classes_cover_irregular_runs():
    st = met.Code.build(PROFILES["r0.1"], 65536, 1).info()
    # 4 checks of degree 11, 1307 of degree 12, 8 checks with (2 + 1), the rest (3 + 1)
    assert st["n_check_classes"] == 4


def test_from_edges_roundtrip_and_sorting():
    vn = [2, 0, 1, 1, 3]
    cn = [1, 0, 0, 1, 1]
    c = met.Code.from_edges(4, 2, vn, cn, [0, 1, 2, 0, 1])
    v, ch, t = c.export()
    np.testing.assert_array_equal(ch, [0, 0, 1, 1, 1])
    # sorted by (check, type, VN)
    np.testing.assert_array_equal(v, [0, 1, 1, 2, 3])
    np.testing.assert_array_equal(t, [1, 2, 0, 0, 1])
    assert c.info()["n_deg1"] == 3


@pytest.mark.parametrize(
    "args,msg",
    [
        ((4, 2, [0, 5], [0, 1]), "out of range"),
        ((4, 1, [0, 0, 1], [0, 0, 0]), "repeated"),
        ((4, 2, [0, 1, 2], [0, 0, 1]), "degree 1"),
    ],
)
def test_from_edges_validation(args, msg):
    with pytest.raises(met.MetError) as e:
        met.Code.from_edges(*args)
    assert e.value.code == -1
    assert msg in str(e.value)


def test_profile_validation():
    bad = Profile("bad", 0.5, vn_types=((0.5, (2, 1)), (0.5, (0, 1))), cn_types=((0.5, (2, 1)), (0.1, (0, 2))))
    with pytest.raises(met.MetError, match="two check types"):
        met.Code.build(bad, 100, 1)
    bad2 = Profile("bad2", 0.5, vn_types=((1.0, (3,)),), cn_types=((0.9, (6,)),))
    with pytest.raises(met.MetError, match="cn_frac"):
        met.Code.build(bad2, 1000, 1)
    with pytest.raises(met.MetError):
        met.Code.build(PROFILES["r0.1"], 1, 1)


def test_edge_count_limited_to_int32_before_allocating():
    """Edge positions are int32: a code with more than 2^31 - 1 edges (the
    rate-0.1 profile at N = 2^30 has about 4.0e9) is refused before any socket
    list is built, and so is a variable degree past the documented bound."""
    with pytest.raises(met.MetError, match="exceed the int32 edge index") as e:
        met.Code.build(PROFILES["r0.1"], 2 ** 30, 1)
    assert e.value.code == -1
    huge = Profile("huge", 0.5, vn_types=((0.5, (70000, 0)), (0.5, (0, 1))), cn_types=((0.5, (0, 1)),))
    with pytest.raises(met.MetError, match="VN degree"):
        met.Code.build(huge, 100, 1)


def test_decode_argument_validation_without_gpu():
    """Validation happens before any HIP call, so it works on a GPU-less host."""
    c = met.Code.build(PROFILES["r0.1"], 4096, 1)
    L = _lib.lib
    P = ctypes.c_void_p
    dummy = P(256)
    n = ctypes.c_size_t()
    assert L.met_decode_workspace_bytes(c.handle, 0, 0, 0, ctypes.byref(n)) == -1
    assert L.met_decode_workspace_bytes(c.handle, 64, 32, 0, ctypes.byref(n)) == -1
    assert L.met_decode_workspace_bytes(None, 64, 0, 0, ctypes.byref(n)) == -1
    assert L.met_decode_workspace_bytes(c.handle, 64, 0, 0, ctypes.byref(n)) == 0 and n.value > 0
    big = n.value
    args = dict(llr=dummy, syn=dummy, B=64, it=10, flags=0, bits=dummy, iters=dummy, conv=dummy, post=None,
                ws=dummy, wsb=big)

    def call(**kw):
        a = dict(args, **kw)
        return L.met_decode(c.handle, a["llr"], a["syn"], a["B"], a["it"], a["flags"], a["bits"], a["iters"],
                            a["conv"], a["post"], a["ws"], a["wsb"], None)

    assert call(B=0) == -1
    assert call(it=0) == -1
    assert call(llr=None) == -1
    assert call(llr=P(258)) == -1          # misaligned float buffer
    assert call(ws=P(264)) == -1           # workspace not 256-byte aligned
    assert call(wsb=big - 1) == -1         # too small
    assert call(flags=64) == -1            # first unknown flag
    assert "flags" in L.met_last_error().decode()
    assert call(flags=_lib.MET_CHECK_LUT) == -1   # the table-driven update needs 8-bit storage
    assert "MET_C2V_Q8" in L.met_last_error().decode()
    assert call(flags=4) == -1             # the all-VN layout needs a larger workspace
    assert "workspace" in L.met_last_error().decode()
    assert L.met_syndrome(c.handle, None, 1, dummy, None) == -1
    assert L.met_syndrome(c.handle, dummy, 0, dummy, None) == -1


def test_workspace_grows_with_batch_and_posterior():
    c = met.Code.build(PROFILES["r0.05"], 8192, 3)
    a = met.workspace_bytes(c, 1)
    b = met.workspace_bytes(c, 64)
    d = met.workspace_bytes(c, 64, posterior=True)
    assert a < b < d


def test_all_vn_layout_sizes():
    """MET_NO_DEG1_SKIP decodes on a layout where degree-1 variable nodes are
    message nodes: every edge is a message edge and every node has a
    posterior row, so its workspace is larger; the code itself is unchanged."""
    c = met.Code.build(PROFILES["r0.1"], 8192, 3)
    info = c.info()
    a = met.workspace_bytes(c, 64)
    b = met.workspace_bytes(c, 64, deg1_skip=False)
    assert b > a
    assert met.workspace_bytes(c, 64, deg1_skip=False) == b  # the view is built once and kept
    assert c.info() == info
    # the extra bytes are at least the degree-1 nodes' check messages and rows
    assert b - a >= 64 * 4 * info["n_deg1"]


def test_fp16_messages_flag():
    """MET_C2V_FP16 halves the message array and needs groups of 64 frames."""
    code = met.Code.build(PROFILES["r0.1"], 4096, 5)
    with pytest.raises(met.MetError):
        met.workspace_bytes(code, 32, c2v_fp16=True)
    info = code.info()
    full, half = met.workspace_bytes(code, 64), met.workspace_bytes(code, 64, c2v_fp16=True)
    assert full - half >= 2 * 64 * info["n_msg_edges"] - 4096


def test_free_is_idempotent():
    c = met.Code.build(PROFILES["r0.02"], 2048, 3)
    c.close()
    c.close()
    _lib.lib.met_code_free(None)


def test_batched_argument_validation_without_gpu():
    c1 = met.Code.build(PROFILES["r0.1"], 4096, 1)
    c2 = met.Code.build(PROFILES["r0.02"], 3000, 2)
    L = _lib.lib
    P = ctypes.c_void_p
    jobs = (_lib.met_job * 2)()
    for k, (c, b) in enumerate(((c1, 64), (c2, 100))):
        jobs[k].code = c.handle
        jobs[k].llr = jobs[k].syn = jobs[k].bits = jobs[k].iters = jobs[k].converged = 256
        jobs[k].B = b
        jobs[k].max_iter = 20
    n = ctypes.c_size_t()
    assert L.met_batched_workspace_bytes(jobs, 2, ctypes.byref(n)) == 0
    both = n.value
    assert L.met_batched_workspace_bytes(jobs, 1, ctypes.byref(n)) == 0 and 0 < n.value < both
    # each job's part is at least what met_decode needs for the same frames
    assert both >= met.workspace_bytes(c1, 64) + met.workspace_bytes(c2, 100)
    assert L.met_batched_workspace_bytes(jobs, 0, ctypes.byref(n)) == -1
    jobs[1].posterior = 256
    assert L.met_batched_workspace_bytes(jobs, 2, ctypes.byref(n)) == -1
    assert "posterior" in L.met_last_error().decode()
    jobs[1].posterior = None
    jobs[1].flags = 8
    assert L.met_batched_workspace_bytes(jobs, 2, ctypes.byref(n)) == -1
    jobs[1].flags = 0
    jobs[0].B = 0
    assert L.met_batched_workspace_bytes(jobs, 2, ctypes.byref(n)) == -1
    jobs[0].B = 64
    jobs[0].llr = 258
    assert L.met_decode_batched(jobs, 2, P(256), both, None, None) == -1
    jobs[0].llr = 256
    assert L.met_decode_batched(jobs, 2, P(264), both, None, None) == -1   # workspace misaligned
    assert L.met_decode_batched(jobs, 2, P(256), both - 1, None, None) == -1
    t = _lib.met_tuning()
    t.check_steps_per_wave = 3
    assert L.met_decode_batched(jobs, 2, P(256), both, ctypes.byref(t), None) == -1
    t.check_steps_per_wave = 0
    t.batch_flags = 64   # first unknown flag
    assert L.met_decode_batched(jobs, 2, P(256), both, ctypes.byref(t), None) == -1
    assert "batch_flags" in L.met_last_error().decode()
    for f in ((_lib.MET_BATCH_KIND_STREAMS | _lib.MET_BATCH_JOB_STREAMS),
              (_lib.MET_BATCH_JOB_STREAMS | _lib.MET_BATCH_JOBS_IN_TURN),
              (_lib.MET_BATCH_KIND_STREAMS | _lib.MET_BATCH_JOBS_IN_TURN)):
        t.batch_flags = f
        assert L.met_decode_batched(jobs, 2, P(256), both, ctypes.byref(t), None) == -1
        assert "exclude" in L.met_last_error().decode()
    assert L.met_batched_check(None, None) == -1


def test_batched_autotune_validation_without_gpu():
    c = met.Code.build(PROFILES["r0.1"], 4096, 1)
    L = _lib.lib
    jobs = (_lib.met_job * 1)()
    jobs[0].code = c.handle
    jobs[0].llr = jobs[0].syn = jobs[0].bits = jobs[0].iters = jobs[0].converged = 256
    jobs[0].B = 64
    jobs[0].max_iter = 20
    n = ctypes.c_size_t()
    assert L.met_batched_workspace_bytes(jobs, 1, ctypes.byref(n)) == 0
    best = _lib.met_tuning()
    ms = ctypes.c_float()
    P = ctypes.c_void_p
    assert L.met_batched_autotune(jobs, 1, P(256), n.value, 0, None, ctypes.byref(ms), None) == -1
    assert L.met_batched_autotune(jobs, 1, P(256), n.value, -1, ctypes.byref(best), None, None) == -1
    assert L.met_batched_autotune(jobs, 1, P(264), n.value, 0, ctypes.byref(best), None, None) == -1
    assert L.met_batched_autotune(jobs, 1, P(256), n.value - 1, 0, ctypes.byref(best), None, None) == -1
    assert L.met_batched_autotune(jobs, 0, P(256), n.value, 0, ctypes.byref(best), None, None) == -1


def test_mdr_argument_validation_without_gpu():
    """Front-end entry points validate before any HIP call."""
    L = _lib.lib
    P = ctypes.c_void_p
    d16, d8 = P(4096), P(4096 + 8)
    assert L.met_mdr_bob(d16, d16, 2, 64, 3, d16, d16, None) == -1        # dimension
    assert "dimension" in L.met_last_error().decode()
    assert L.met_mdr_bob(d16, d16, 2, 60, 8, d16, d16, None) == -1        # N not a multiple of d
    assert L.met_mdr_bob(d16, d16, 0, 64, 8, d16, d16, None) == -1        # B
    assert L.met_mdr_bob(None, d16, 2, 64, 8, d16, d16, None) == -1       # NULL
    assert L.met_mdr_bob(d8, d16, 2, 64, 8, d16, d16, None) == -1         # y not 16-byte aligned
    assert L.met_mdr_bob(d16, P(4097), 2, 64, 8, d16, d16, None) == -1    # bits not 8-byte aligned
    assert L.met_mdr_bob(d16, d16, 1 << 20, 1 << 20, 8, d16, d16, None) == -1  # B N above 2^36
    assert L.met_mdr_alice(d16, d16, d16, 0.0, 2, 64, 8, d16, None) == -1     # sigma^2 <= 0
    assert L.met_mdr_alice(d16, d16, d16, float("nan"), 2, 64, 8, d16, None) == -1
    assert L.met_mdr_alice(d16, d8, d16, 1.0, 2, 64, 8, d16, None) == -1      # alpha misaligned
    assert L.met_mdr_alice(d16, d16, d16, 1.0, 2, 64, 5, d16, None) == -1     # dimension


def test_noalloc_validation_without_gpu():
    """The allocation-free decode refuses what it cannot do before any HIP call."""
    c = met.Code.build(PROFILES["r0.1"], 4096, 1)
    L = _lib.lib
    dummy = ctypes.c_void_p(256)
    assert L.met_decode_noalloc(None, dummy, dummy, 4, 10, 0, dummy, dummy, dummy, None, None) == -1
    assert L.met_decode_noalloc(c.handle, dummy, dummy, 0, 10, 0, dummy, dummy, dummy, None, None) == -1
    assert L.met_decode_noalloc(c.handle, dummy, dummy, 4, 10, 4, dummy, dummy, dummy, None, None) == -1
    assert "MET_NO_DEG1_SKIP" in L.met_last_error().decode()
    n = ctypes.c_size_t()
    assert L.met_decode_workspace_bytes(c.handle, 60000, 0, 0, ctypes.byref(n)) == 0
    assert n.value > _lib.MET_NOALLOC_SCRATCH_BYTES
    assert L.met_decode_noalloc(c.handle, dummy, dummy, 60000, 10, 0, dummy, dummy, dummy, None, None) == -1
    assert "scratch" in L.met_last_error().decode()


@pytest.mark.parametrize("name,n,seed,depth", [("r0.1", 4096, 1, None), ("r0.05", 4096, 2, None),
                                               ("r0.02", 4096, 3, None), ("r0.1", 8192, 4, [4, 1, 1]),
                                               ("r0.02", 8192, 5, [2, 2, 1])])
def test_cpp_peg_matches_oracle(name, n, seed, depth):
    """The C++ progressive-edge-growth builder equals oracle/peg.py bit for bit."""
    from oracle import peg

    cg = met.Code.build_peg(PROFILES[name], n, seed, depth)
    vn, cn, et = cg.export()
    co = peg.build(PROFILES[name], n, seed, depth)
    np.testing.assert_array_equal(vn, co.v)
    np.testing.assert_array_equal(cn, co.c)
    np.testing.assert_array_equal(et, co.t)


def test_peg_validation():
    with pytest.raises(met.MetError, match="depth"):
        met.Code.build_peg(PROFILES["r0.1"], 4096, 1, [0, 1, 1])
    with pytest.raises(met.MetError, match="depth"):
        met.Code.build_peg(PROFILES["r0.1"], 4096, 1, [17, 1, 1])


def test_q8_messages_flag():
    c = met.Code.build(PROFILES["r0.1"], 4096, 1)
    L = _lib.lib
    n = ctypes.c_size_t()
    assert L.met_decode_workspace_bytes(c.handle, 64, _lib.MET_C2V_Q8, 0, ctypes.byref(n)) == 0
    q8 = n.value
    assert L.met_decode_workspace_bytes(c.handle, 64, _lib.MET_C2V_FP16, 0, ctypes.byref(n)) == 0
    assert q8 < n.value
    assert L.met_decode_workspace_bytes(c.handle, 20, _lib.MET_C2V_Q8, 0, ctypes.byref(n)) == -1   # W < 64
    assert L.met_decode_workspace_bytes(c.handle, 64, _lib.MET_C2V_Q8 | _lib.MET_C2V_FP16, 0,
                                        ctypes.byref(n)) == -1


def test_batched_decoder_rejects_unknown_stream_modes():
    with pytest.raises(ValueError, match="streams"):
        met.BatchedDecoder(streams="parallel")
    for mode, flag in (("one", 0), ("kinds", _lib.MET_BATCH_KIND_STREAMS), ("jobs", _lib.MET_BATCH_JOB_STREAMS),
                       ("serial", _lib.MET_BATCH_JOBS_IN_TURN)):
        d = met.BatchedDecoder(streams=mode, stagger=False)
        assert d.tuning.batch_flags == flag | _lib.MET_BATCH_NO_STAGGER
