#!/usr/bin/env python3
"""Writes large_oracle.json: the oracle's HEGMM-En result for the large
workload (A 128x96 times B 96x128, entries in [-4, 4], BGV N = 32768,
t = 786433, 8 + 2 primes), as SHA-256 digests of the canonical words of the
packed operands and of the result plus a few sampled words.

Calls only oracle/ and the seeded input generators; takes minutes on a
multi-core host.  Usage: python tests/golden/make_large_golden.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import bgv, hegmm as H  # noqa: E402
from oracle.ring import Params  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_oracle.json")


def digest(words: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


def main():
    c = workloads.LARGE
    m, l, n = 128, 96, 128
    nonce = 1
    A, B = workloads.large_operands()
    P = Params(c.N, c.t, c.L, c.alpha)
    t0 = time.time()
    ks = bgv.KeySet(P, c.seed, H.galois_elements(P, [(m, l, n)]))
    print(f"keys: {len(ks.rot)} rotation keys in {time.time() - t0:.0f} s", flush=True)
    pl = H.plan(m, l, n, P.S)
    ox = H.encrypt_operand(ks, pl, 0, A, B, nonce)
    oy = H.encrypt_operand(ks, pl, 1, A, B, nonce)
    t1 = time.time()
    res = H.hegmm(ks, pl, ox, oy, H.MaskCache(P))
    print(f"hegmm: {time.time() - t1:.0f} s", flush=True)
    words = H.export_d7(res)
    C = H.decrypt_result(ks, pl, res)
    assert np.array_equal(C, workloads.plain_matmul_mod(A, B, c.t)), "oracle result does not decrypt to A.B"
    rng = np.random.default_rng(7)
    idx = sorted(int(i) for i in rng.choice(words.size, size=16, replace=False))
    doc = {
        "workload": "HEGMM-En A(128x96) x B(96x128), entries in [-4,4], BGV N=32768 t=786433 L=8 alpha=2",
        "seed": c.seed, "nonce": nonce, "shape": [m, l, n],
        "left_operand_sha256": digest(np.concatenate([H.export_d7(x) for x in ox])),
        "right_operand_sha256": digest(np.concatenate([H.export_d7(y) for y in oy])),
        "result_words": int(words.size),
        "result_sha256": digest(words),
        "result_samples": {str(i): int(words[i]) for i in idx},
        "generator": "tests/golden/make_large_golden.py (oracle only)",
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
