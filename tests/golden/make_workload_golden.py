#!/usr/bin/env python3
"""Writes batched_oracle.json and serving_oracle.json: SHA-256 digests of the
oracle's HEGMM-En result (canonical words) for every request of two whole
workloads, so that GPU tests can compare every result, not a sample.

* batched: all 256 requests of workloads.batched_requests(256) (BGV N = 8192,
  t = 65537, 4 + 1 primes; shapes uniform over {8, ..., 64}^3), operands of
  request i encrypted with nonce i;
* serving: the first 64 requests of workloads.serving_requests (BGV N = 16384,
  t = 65537, 6 + 2 primes; shapes over {16, ..., 128}^3 capped by the slot
  count), operands of request i encrypted with nonce i.

Every oracle result is also decrypted and checked against the brute-force
product.  Calls only oracle/ and the seeded input generators; the requests
are spread over worker processes (each builds the keys its requests need).
Usage: python tests/golden/make_workload_golden.py [batched|serving] [workers]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
SERVING_COUNT = 64


def digest(words: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


def _requests(name):
    import workloads
    if name == "batched":
        return workloads.BATCHED, [(m, l, n, A, B) for (m, l, n, A, B) in workloads.batched_requests(256)]
    return workloads.SERVING, [(m, l, n, A, B) for (_, m, l, n, A, B) in workloads.serving_requests(SERVING_COUNT)]


def _work(arg):
    name, idx = arg
    import workloads
    from oracle import bgv, hegmm as H
    from oracle.ring import Params
    cfg, reqs = _requests(name)
    P = Params(cfg.N, cfg.t, cfg.L, cfg.alpha)
    ks = bgv.KeySet(P, cfg.seed, H.galois_elements(P, [reqs[i][:3] for i in idx]))
    masks = H.MaskCache(P)
    out = {}
    for i in idx:
        m, l, n, A, B = reqs[i]
        pl = H.plan(m, l, n, P.S)
        res = H.hegmm(ks, pl, H.encrypt_operand(ks, pl, 0, A, B, i), H.encrypt_operand(ks, pl, 1, A, B, i), masks)
        assert np.array_equal(H.decrypt_result(ks, pl, res), workloads.plain_matmul_mod(A, B, cfg.t)), i
        out[i] = digest(H.export_d7(res))
    return out


def make(name, workers):
    import multiprocessing as mp
    cfg, reqs = _requests(name)
    # spread requests of similar cost over the workers, keep shapes together
    order = sorted(range(len(reqs)), key=lambda i: (reqs[i][0] * reqs[i][1] * reqs[i][2], i))
    parts = [order[w::workers] for w in range(workers)]
    t0 = time.time()
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        got = {}
        for d in pool.imap_unordered(_work, [(name, p) for p in parts]):
            got.update(d)
            print(f"{name}: {len(got)}/{len(reqs)} in {time.time() - t0:.0f} s", flush=True)
    doc = {
        "workload": name,
        "ring": {"N": cfg.N, "t": cfg.t, "L": cfg.L, "alpha": cfg.alpha},
        "seed": cfg.seed,
        "nonce": "request index",
        "requests": [{"shape": list(reqs[i][:3]), "result_sha256": got[i]} for i in range(len(reqs))],
        "generator": "tests/golden/make_workload_golden.py (oracle only)",
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {path}")


if __name__ == "__main__":
    which = sys.argv[1:2] or ["batched", "serving"]
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    for name in (["batched", "serving"] if which == ["all"] else which):
        make(name, workers)
