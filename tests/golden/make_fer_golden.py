"""Writes the oracle's per-frame outcomes used by the GPU FER-parity test.

    python tests/golden/make_fer_golden.py [--frames 1024] [--workers 8] [--construction peg]

Calls only the FP64 oracle (`oracle/`) and the seeded input module
(`met_inputs`).  For each rate: the code built from the profile with CODE_SEED
at N = 65536 by `oracle.code.build` (the seeded random construction; files
fer_<rate>_N65536.json) or by `oracle.peg.build` at its default depths
(progressive edge growth; files fer_peg_<rate>_N65536.json), frames
FRAME_SEED + f at the waterfall SNR, decoded in early-exit mode with the
rate's iteration budget.  Stored per frame: converged flag, iterations, frame
error (decoded bits != sent bits) and the SHA-1 of the decoded bits.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from met_inputs import ITER_BUDGET, PROFILES, WATERFALL_SNR, make_frames  # noqa: E402
from oracle import bp, code as oc, peg  # noqa: E402

N = 65536
CODE_SEED = 31
FRAME_SEED = 90000
CHUNK = 16
_CODE = {}


def _work(args):
    prof, f0, nf = args
    code = _CODE[prof]
    bits, llr = make_frames(N, nf, WATERFALL_SNR[prof], FRAME_SEED, first_frame=f0)
    syn = oc.syndrome(code, bits)
    r = bp.decode(code, llr, syn, ITER_BUDGET[prof])
    out = []
    for i in range(nf):
        out.append({
            "frame": f0 + i,
            "converged": int(r.converged[i]),
            "iterations": int(r.iterations[i]),
            "frame_error": int(np.any(r.bits[i] != bits[i])),
            "bits_sha1": hashlib.sha1(r.bits[i].tobytes()).hexdigest(),
        })
    return out


def code_sha1(code) -> str:
    """SHA-1 of the edge list (variable, check, type as int64, in the code's
    (check, type, variable) order): lets a test check that another builder made
    exactly this graph."""
    h = hashlib.sha1()
    for a in (code.v, code.c, code.t):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=1024)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--rates", default="r0.1,r0.05,r0.02")
    ap.add_argument("--construction", choices=("random", "peg"), default="random")
    ap.add_argument("--add-code-hash", action="store_true",
                    help="only build each code and store its edge-list SHA-1 in the existing file")
    args = ap.parse_args()
    for prof in args.rates.split(","):
        if args.construction == "peg":
            _CODE[prof] = peg.build(PROFILES[prof], N, CODE_SEED)
        else:
            _CODE[prof] = oc.build(PROFILES[prof], N, CODE_SEED)
        stem = "fer_peg_%s_N%d.json" if args.construction == "peg" else "fer_%s_N%d.json"
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), stem % (prof, N))
        if args.add_code_hash:
            with open(path) as f:
                rec = json.load(f)
            assert rec["code_seed"] == CODE_SEED and rec["N"] == N
            rec["code_sha1"] = code_sha1(_CODE[prof])
            with open(path, "w") as f:
                json.dump(rec, f, separators=(",", ":"))
            print(prof, "code_sha1", rec["code_sha1"], "->", path, flush=True)
            continue
        jobs = [(prof, f0, min(CHUNK, args.frames - f0)) for f0 in range(0, args.frames, CHUNK)]
        with mp.get_context("fork").Pool(args.workers) as pool:
            frames = [x for part in pool.map(_work, jobs) for x in part]
        rec = {
            "source": "oracle/bp.py early-exit decode; tests/golden/make_fer_golden.py",
            "construction": args.construction,
            "peg_depth": peg.default_depths(PROFILES[prof]) if args.construction == "peg" else None,
            "profile": prof,
            "code_sha1": code_sha1(_CODE[prof]),
            "N": N,
            "code_seed": CODE_SEED,
            "frame_seed": FRAME_SEED,
            "snr": WATERFALL_SNR[prof],
            "max_iter": ITER_BUDGET[prof],
            "frames": frames,
        }
        with open(path, "w") as f:
            json.dump(rec, f, separators=(",", ":"))
        fer = sum(x["frame_error"] for x in frames) / len(frames)
        print(prof, "FER", fer, "converged", sum(x["converged"] for x in frames), "->", path, flush=True)


if __name__ == "__main__":
    main()
