"""CPU oracle for the HE matrix multiplication path (TEST INFRASTRUCTURE).

A plain, slow, obviously correct model of what the GPU library computes:
BGV over RNS with hybrid key switching, and the paper's HEGMM-En algorithm
(Algorithm 2) composed from its SIMD primitives.  Only `tests/`, the smoke
check in `__graft_entry__` and the CPU-baseline leg of `bench.py` may import
it.  It shares no code with the GPU library (`paper_2405_02238_amd`), and the
library never imports it.

Layout:
  bgv_ref.c  C: 128-bit-product modular arithmetic, the negacyclic transform,
             SplitMix64 streams, samplers, digit lift and the division by P
  ring.py    parameters (primes, roots, zeta_t, Gaussian table), row-wise ops,
             slot encoding
  bgv.py     keys, encryption, decryption, the primitives and key switching
  hegmm.py   planning, packing, the HEGMM-En loop, unpacking

Pinning (what checks the oracle against something other than itself) is in
tests/test_oracle_*.py.  Ciphertext bits of key switching, rotation and
relinearisation are fixed by the conventions in the design notes, not by the
paper ("parity unpinned" by the paper for those bits; decryption of every
result is pinned by brute-force matrix products).
"""
from . import ring, bgv, hegmm  # noqa: F401
from .ring import Params  # noqa: F401
