"""Write the full-size oracle references used by the GPU parity tests.

Test infrastructure: this script calls only the FP64 CPU oracle (``oracle/``)
and the seeded input generators (``paper_2503_23385_amd/workloads.py``); no
value in the files it writes comes from the GPU path.

For each workload it stores, in ``oracle_<name>.npz``:

- ``R``: the oracle's R of the join matrix (N x N, rows normalised to a
  non-negative diagonal), i.e. the Householder QR of the compact matrix of
  Claim 1 (Section 1), and ``sigma``: its singular values by one-sided Jacobi;
- for the batch, ``R_<i>`` / ``sigma_<i>`` for every instance i;
- ``input_sha1``: a digest of the generated inputs, so that a test can tell a
  stale reference (a changed generator) from a wrong GPU result.

Usage: ``python tests/golden/make_golden.py [cfg1 cfg2 cfg3 cfg4 cfg5]``.
About two minutes on 8 host cores for all five.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2503_23385_amd import workloads as W  # noqa: E402


def input_digest(insts) -> str:
    h = hashlib.sha1()
    for inst in insts:
        for X in (inst.A, inst.B, inst.keys_A, inst.keys_B):
            if X is None:
                h.update(b"none")
            else:
                h.update(str(X.dtype).encode())
                h.update(str(X.shape).encode())
                h.update(np.ascontiguousarray(X).tobytes())
    return h.hexdigest()


def path_for(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def instances(name: str):
    if name == "cfg4":
        return W.config4()
    return [W.CONFIGS[int(name[3:])]()]


def write(name: str) -> None:
    t0 = time.perf_counter()
    insts = instances(name)
    out = {"input_sha1": np.array(input_digest(insts))}
    for i, inst in enumerate(insts):
        R = oracle.r(inst)
        S = oracle.sigma(R)
        key = "" if len(insts) == 1 else f"_{i}"
        out["R" + key] = R
        out["sigma" + key] = S
    out["count"] = np.array(len(insts))
    np.savez_compressed(path_for(name), **out)
    print(f"{name}: {len(insts)} instance(s), {time.perf_counter() - t0:.1f} s -> {path_for(name)}", flush=True)


def load(name: str):
    """Stored references: (list of (R, sigma) per instance, input digest)."""
    with np.load(path_for(name), allow_pickle=False) as z:
        count = int(z["count"])
        if count == 1:
            refs = [(z["R"], z["sigma"])]
        else:
            refs = [(z[f"R_{i}"], z[f"sigma_{i}"]) for i in range(count)]
        return refs, str(z["input_sha1"])


if __name__ == "__main__":
    names = sys.argv[1:] or ["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"]
    for nm in names:
        write(nm)
