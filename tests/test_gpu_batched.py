"""Batched decoding: every job's outputs equal met_decode's.

The batched launch runs the same check and variable updates as met_decode
(Methods, Steps 3-5) for several jobs at once, interleaved phase by phase
inside one persistent kernel or one launch per phase.  Its results must not
differ in a single bit or iteration count from decoding each job on its own,
for any launch shape.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from met_inputs import PROFILES, make_frames  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _job(prof, n, b, snr, max_iter, seed, fixed=False):
    code = met.Code.build(PROFILES[prof], n, seed)
    bits, llr = make_frames(n, b, snr, 700 + seed)
    d_bits = torch.from_numpy(bits).to(DEV)
    syn = met.syndrome(code, d_bits)
    return met.Job(code, torch.from_numpy(llr).to(DEV), syn, max_iter, fixed), bits


@pytest.fixture(scope="module")
def mix():
    # three rates, ragged batch sizes (one, two and three groups of 64 frames)
    # and both stopping rules
    return [
        _job("r0.1", 16384, 64, 0.19, 30, 1),
        _job("r0.05", 12000, 100, 0.10, 40, 2),
        _job("r0.02", 9000, 30, 0.065, 50, 3),
        _job("r0.1", 5000, 130, 0.22, 7, 4, fixed=True),
    ]


def _plain(jobs):
    return [met.decode(j.code, j.llr, j.syn, j.max_iter, fixed_iters=j.fixed_iters) for j in jobs]


def _same(a, b, tag):
    for k, (x, y) in enumerate(zip(a, b)):
        np.testing.assert_array_equal(x.iterations.cpu().numpy(), y.iterations.cpu().numpy(), err_msg="%s job %d" % (tag, k))
        np.testing.assert_array_equal(x.converged.cpu().numpy(), y.converged.cpu().numpy(), err_msg="%s job %d" % (tag, k))
        np.testing.assert_array_equal(x.bits.cpu().numpy(), y.bits.cpu().numpy(), err_msg="%s job %d" % (tag, k))


@pytest.mark.parametrize("tuning", [dict(), dict(check_steps_per_wave=1), dict(check_steps_per_wave=2),
                                    dict(stagger=False), dict(graph=False), dict(blocks_per_cu=1),
                                    dict(interleave=32), dict(interleave=16), dict(interleave=16, graph=False),
                                    dict(phase_launches=True), dict(phase_launches=True, stagger=False),
                                    dict(phase_launches=True, check_steps_per_wave=2),
                                    dict(phase_launches=True, check_steps_per_wave=1, graph=False),
                                    dict(phase_launches=True, interleave=32),
                                    dict(phase_launches=True, interleave=16, stagger=False),
                                    dict(streams="kinds"), dict(streams="kinds", stagger=False),
                                    dict(streams="kinds", graph=False, interleave=32),
                                    dict(streams="jobs"), dict(streams="jobs", stagger=False, check_steps_per_wave=2),
                                    dict(streams="jobs", graph=False), dict(streams="jobs", interleave=16),
                                    dict(streams="serial"), dict(streams="serial", graph=False, stagger=False)])
def test_batched_equals_plain_decode(mix, tuning):
    jobs = [j for j, _ in mix]
    print("batched", tuning, flush=True)
    ref = _plain(jobs)
    dec = met.BatchedDecoder(**tuning)
    out = dec(jobs)
    torch.cuda.synchronize()
    assert not dec.barrier_expired()
    _same(out, ref, str(tuning))
    # the fixed-iteration job ran its whole budget; early-exit jobs converged mostly
    assert np.all(out[3].iterations.cpu().numpy() == 7)
    assert out[0].converged.cpu().numpy().mean() > 0.3


@pytest.mark.parametrize("tuning", [dict(phase_launches=True, stagger=False), dict(streams="kinds"),
                                    dict(streams="jobs", stagger=False), dict(streams="serial", graph=False)])
def test_jobs_whose_checks_fill_the_gpu(tuning):
    """Jobs large enough that their (3,1) / (2,1) check classes take launches
    of their own (the plain decoder's check kernels) next to a small job that
    shares the batched launch: every output equals the plain decode's."""
    jobs = [_job("r0.1", 65536, 64, 0.19, 24, 51)[0], _job("r0.05", 65536, 64, 0.10, 18, 52)[0],
            _job("r0.02", 9000, 24, 0.065, 30, 53)[0]]
    print("large jobs", tuning, flush=True)
    out = met.BatchedDecoder(**tuning)(jobs)
    torch.cuda.synchronize()
    _same(out, _plain(jobs), str(tuning))


def test_graph_replay_and_reuse_of_outputs(mix):
    jobs = [j for j, _ in mix]
    ref = _plain(jobs)
    dec = met.BatchedDecoder()
    out = dec(jobs)
    for rep in range(3):
        for o in out:  # poison the outputs: each replay must rewrite all of them
            o.bits.fill_(7)
            o.iterations.fill_(-1)
            o.converged.fill_(9)
        dec(jobs, outputs=out)
        torch.cuda.synchronize()
        assert not dec.barrier_expired()
        _same(out, ref, "replay %d" % rep)


def test_single_job_and_different_job_sets(mix):
    for sel in ([0], [2, 1], [3, 0, 2]):
        jobs = [mix[k][0] for k in sel]
        print("jobs", sel, flush=True)
        out = met.decode_batched(jobs)
        torch.cuda.synchronize()
        _same(out, _plain(jobs), str(sel))


def test_launch_stops_when_every_frame_has_converged():
    """Jobs whose frames all converge long before their budgets: the launch
    stops at the first barrier after the last frame retired (outputs equal the
    plain decode's, which runs every iteration), also next to a job with more
    work left and next to a fixed-iteration job."""
    easy = [_job("r0.1", 4096, 64, 0.5, 300, 21)[0], _job("r0.02", 4096, 3, 0.2, 400, 22)[0]]
    slow = _job("r0.05", 8192, 20, 0.10, 60, 23)[0]
    fixed = _job("r0.1", 4096, 8, 0.5, 40, 24, fixed=True)[0]
    for sel in (easy, easy + [slow], [fixed] + easy):
        out = met.decode_batched(sel)
        torch.cuda.synchronize()
        ref = _plain(sel)
        _same(out, ref, "stop")
    conv = [o.converged.cpu().numpy() for o in _plain(easy)]
    assert all(c.all() for c in conv)


def test_tree_codes_with_runtime_degree_checks():
    from tests.trees import random_tree
    from oracle import code as oc

    rng = np.random.default_rng(11)
    jobs = []
    for k in range(2):
        n, m, v, c, t = random_tree(40 + 10 * k, rng)
        code_o = oc.from_edges(n, m, v, c, t, n_edge_types=3)
        code = met.Code.from_edges(n, m, v, c, t)
        x = rng.integers(0, 2, (70, n)).astype(np.uint8)
        s = oc.syndrome(code_o, x)
        llr = rng.normal(0.5, 1.5, (70, n)).astype(np.float32)
        jobs.append(met.Job(code, torch.from_numpy(llr).to(DEV), torch.from_numpy(s).to(DEV), 25))
    jobs.append(_job("r0.1", 4096, 64, 0.2, 20, 9)[0])
    ref = _plain(jobs)
    for w in (64, 16):
        out = met.decode_batched(jobs, interleave=w)
        torch.cuda.synchronize()
        _same(out, ref, "trees, interleave %d" % w)
    # schedules where the (3,1) / (2,1) checks have launches of their own keep
    # several steps per wave next to the run-time-degree classes
    for kw in (dict(phase_launches=True, stagger=False), dict(phase_launches=True, stagger=False,
                                                             check_steps_per_wave=2),
               dict(phase_launches=True), dict(streams="kinds"), dict(streams="serial", graph=False),
               dict(streams="jobs", stagger=False)):
        out = met.decode_batched(jobs, **kw)
        torch.cuda.synchronize()
        _same(out, ref, "trees, %s" % kw)


def test_autotuner_picks_a_valid_shape_and_caches_it(mix):
    import time

    jobs = [j for j, _ in mix[:3]]
    dec = met.BatchedDecoder()
    t0 = time.perf_counter()
    shape = dec.autotune(jobs, probe_iters=3)
    t1 = time.perf_counter()
    print("autotuned", shape, "in %.2f s" % (t1 - t0), flush=True)
    assert shape["check_steps_per_wave"] in (1, 2, 4)
    assert shape["interleave"] in (16, 32, 64)
    if shape["schedule"] == "persistent":
        assert 1 <= shape["blocks_per_cu"] <= 6
    else:
        assert shape["schedule"] == "phase launches" and shape["blocks_per_cu"] == 0  # no resident grid
    assert shape["probe_ms"] > 0
    again = met.BatchedDecoder().autotune(jobs, probe_iters=3)
    assert again == shape                     # served from the cache
    assert time.perf_counter() - t1 < 0.5 * (t1 - t0) + 0.05
    out = dec(jobs)
    torch.cuda.synchronize()
    assert not dec.barrier_expired()
    _same(out, _plain(jobs), "autotuned")


def test_graph_cache_does_not_outlive_a_freed_code():
    """Same buffers, sizes and host address for a new code after the old one was
    freed: the cached graph of the old code must not be replayed."""
    n, b = 4096, 64
    d_llr = torch.empty((b, n), dtype=torch.float32, device=DEV)
    outs = None
    dec = met.BatchedDecoder()
    syn_buf = None
    for seed in (31, 32, 33):
        code = met.Code.build(PROFILES["r0.1"], n, seed)
        bits, llr = make_frames(n, b, 0.2, 900 + seed)
        d_llr.copy_(torch.from_numpy(llr))
        syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
        if syn_buf is None:
            syn_buf = syn.clone()
        syn_buf.copy_(syn)
        job = met.Job(code, d_llr, syn_buf, 12)
        outs = dec([job], outputs=outs)
        torch.cuda.synchronize()
        _same(outs, _plain([job]), "seed %d" % seed)
        code.close()


@pytest.mark.parametrize("phase_launches", [False, True])
def test_batched_against_the_oracle_at_waterfall_snrs(phase_launches):
    """One batched launch of three jobs (one per rate, waterfall SNRs, budgets
    60 / 90 / 120; persistent or one launch per phase) against the FP64 oracle
    directly: converged flags are the exact syndrome test of the decoded bits,
    and every frame's word and count (within one iteration) equal the oracle's,
    except where tests/oracle_outcome.py shows the oracle's own outcome to move
    under FP32-sized perturbations (listed)."""
    from oracle import code as oc
    from tests import oracle_outcome as oo

    specs = [("r0.1", 16384, 40, 0.19, 60, 41), ("r0.05", 12000, 33, 0.10, 90, 42),
             ("r0.02", 9000, 24, 0.065, 120, 43)]
    jobs, inputs = [], []
    for prof, n, b, snr, max_iter, seed in specs:
        code = met.Code.build(PROFILES[prof], n, seed)
        bits, llr = make_frames(n, b, snr, 700 + seed)
        code_o = oc.build(PROFILES[prof], n, seed)
        syn = oc.syndrome(code_o, bits)
        jobs.append(met.Job(code, torch.from_numpy(llr).to(DEV), torch.from_numpy(syn).to(DEV), max_iter))
        inputs.append((code_o, llr, syn, max_iter))
    print("batched vs oracle", [s[:5] for s in specs], "phase launches" if phase_launches else "persistent",
          flush=True)
    dec = met.BatchedDecoder(phase_launches=phase_launches)
    out = dec(jobs)
    torch.cuda.synchronize()
    assert not dec.barrier_expired()
    for (code_o, llr, syn, max_iter), o, spec in zip(inputs, out, specs):
        got = o.bits.cpu().numpy(), o.converged.cpu().numpy(), o.iterations.cpu().numpy()
        acc, rep = oo.compare(code_o, llr, syn, max_iter, *got)
        print("  %s: %d of %d frames converged, %d differ from the oracle with proof" % (
            spec[0], int(got[1].sum()), spec[2], len(acc)), flush=True)
        for line in rep:
            print("   ", line, flush=True)
        assert got[1].sum() >= spec[2] // 4
        assert len(acc) <= spec[2] // 10
