"""Decoding without allocation: met_decode_noalloc against met_decode.

The allocation-free entry point runs the same kernels on a fixed device
array inside the library, so its outputs must equal met_decode's bit for bit.
Two calls in a row (the second with a smaller code and fewer frames) check
that nothing the first call leaves in the shared array reaches the second.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from paper_1711_01783_amd._lib import (MET_EINVAL, MET_ESTATE, MET_FIXED_ITERS, MET_NO_DEG1_SKIP,  # noqa: E402
                                       MET_NOALLOC_SCRATCH_BYTES, lib)
from met_inputs import PROFILES, make_frames  # noqa: E402
from oracle import code as oc  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(prof, n, b, snr, seed, code_seed):
    code_o = oc.build(PROFILES[prof], n, code_seed)
    code_g = met.Code.build(PROFILES[prof], n, code_seed)
    bits, llr = make_frames(n, b, snr, seed)
    syn = oc.syndrome(code_o, bits)
    return code_g, torch.from_numpy(llr).to(DEV), torch.from_numpy(syn).to(DEV)


def _outputs(code, b, posterior):
    return (torch.full((b, code.N), 7, dtype=torch.uint8, device=DEV),
            torch.full((b,), -5, dtype=torch.int32, device=DEV),
            torch.full((b,), 9, dtype=torch.uint8, device=DEV),
            torch.full((b, code.N), float("nan"), dtype=torch.float32, device=DEV) if posterior else None)


def _call(code, llr, syn, max_iter, flags, outs):
    bits, iters, conv, post = outs
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.met_decode_noalloc(code.handle, llr.data_ptr(), syn.data_ptr(), int(llr.shape[0]), int(max_iter),
                                  flags, bits.data_ptr(), iters.data_ptr(), conv.data_ptr(),
                                  None if post is None else post.data_ptr(), stream)


def _same(ref, outs):
    bits, iters, conv, post = outs
    np.testing.assert_array_equal(bits.cpu().numpy(), ref.bits.cpu().numpy())
    np.testing.assert_array_equal(iters.cpu().numpy(), ref.iterations.cpu().numpy())
    np.testing.assert_array_equal(conv.cpu().numpy(), ref.converged.cpu().numpy())
    if post is not None:
        np.testing.assert_array_equal(post.cpu().numpy(), ref.posterior.cpu().numpy())


@pytest.mark.parametrize("fixed,posterior,max_iter", [(False, False, 60), (True, True, 12)])
def test_noalloc_equals_decode_two_calls(fixed, posterior, max_iter):
    # first a larger input (one group of 64 frames at N = 16384), then a
    # smaller code with fewer frames (groups of 16 at N = 4096)
    big = _inputs("r0.1", 16384, 40, 0.21, 31, 7)
    small = _inputs("r0.02", 4096, 5, 0.07, 32, 8)
    print("noalloc: fixed=%s posterior=%s max_iter=%d" % (fixed, posterior, max_iter), flush=True)
    refs = [met.decode(c, l, s, max_iter, fixed_iters=fixed, posterior=posterior) for c, l, s in (big, small)]
    torch.cuda.synchronize()
    flags = MET_FIXED_ITERS if fixed else 0
    outs = [_outputs(c, int(l.shape[0]), posterior) for c, l, _ in (big, small)]
    for (c, l, s), o in zip((big, small), outs):
        rc = _call(c, l, s, max_iter, flags, o)
        assert rc == 0, lib.met_last_error().decode()
    torch.cuda.synchronize()
    for ref, o in zip(refs, outs):
        _same(ref, o)
    if not fixed:  # the early-exit case must have frames that stopped early
        assert (refs[0].iterations < max_iter).any()


def test_noalloc_refusals():
    code, llr, syn = _inputs("r0.1", 4096, 4, 0.25, 33, 9)
    outs = _outputs(code, 4, False)
    # the adjacency is not on the device yet: uploading it would allocate
    assert _call(code, llr, syn, 10, 0, outs) == MET_ESTATE
    met.syndrome(code, torch.zeros((4, code.N), dtype=torch.uint8, device=DEV))
    torch.cuda.synchronize()
    assert _call(code, llr, syn, 10, 0, outs) == 0
    # a second layout of the code would be built (allocation)
    assert _call(code, llr, syn, 10, MET_NO_DEG1_SKIP, outs) == MET_EINVAL
    # more frames than the fixed array holds: refused before anything runs
    need = met.workspace_bytes(code, 60000)
    assert need > MET_NOALLOC_SCRATCH_BYTES
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.met_decode_noalloc(code.handle, llr.data_ptr(), syn.data_ptr(), 60000, 10, 0, outs[0].data_ptr(),
                                outs[1].data_ptr(), outs[2].data_ptr(), None, stream)
    assert rc == MET_EINVAL and "scratch" in lib.met_last_error().decode()
    torch.cuda.synchronize()
