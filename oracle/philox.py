"""Philox-4x32-10 counter-based generator, written from its published definition.

Source of the definition: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11.  The paper's method
only asks for i.i.d. unit Gaussian noise per cell (Sec. 2, step 1; Sec. 2.1
names SPRNG, which is not available here); a counter-based generator makes
every cell reproducible from (seed, cell index) alone.

Definition used here (one Philox-4x32 bijection, 10 rounds):

* state: four 32-bit words (x0, x1, x2, x3) = the counter; key (k0, k1).
* one round: multiply x0 by M0 and x2 by M1 as 32x32 -> 64-bit products,
  split each product into its high and low 32-bit halves (h0, l0), (h1, l1),
  and form the new state (h1 ^ x1 ^ k0, l1, h0 ^ x3 ^ k1, l0).
* key schedule: the key used in round r is (k0 + r*W0, k1 + r*W1) mod 2^32.
* multipliers M0 = 0xD2511F53, M1 = 0xCD9E8D57 and Weyl increments
  W0 = 0x9E3779B9 (golden ratio), W1 = 0xBB67AE85 (sqrt(3) - 1), as chosen
  in that paper.

Pins (tests/test_oracle_philox.py): the one-round and two-round outputs for
counters with a single non-zero word reduce to closed forms of the round
(which word each product lands in, which key word enters where); each round is
inverted independently (odd multipliers are invertible mod 2^32) and must
give the counter back; zero rounds is the identity; output bits are balanced,
bytes pass a chi-square test, and a one-bit counter change flips about half of
the output bits.  No published known-answer vectors are available here, so
the full 10-round outputs are pinned only through these properties.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
ROUNDS = 10
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32(ctr, key, rounds=ROUNDS):
    """Apply the Philox-4x32 bijection.

    ctr: tuple of four arrays (or ints) of 32-bit counter words.
    key: tuple of two 32-bit key words.
    Returns a tuple of four numpy uint64 arrays holding 32-bit words.
    All products fit in uint64 exactly (both factors < 2^32).
    """
    x0, x1, x2, x3 = (np.asarray(w, dtype=np.uint64) & _MASK for w in ctr)
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for _ in range(rounds):
        p0 = m0 * x0
        p1 = m1 * x2
        h0, l0 = p0 >> np.uint64(32), p0 & _MASK
        h1, l1 = p1 >> np.uint64(32), p1 & _MASK
        x0, x1, x2, x3 = h1 ^ x1 ^ k0, l1, h0 ^ x3 ^ k1, l0
        k0 = (k0 + np.uint64(W0)) & _MASK
        k1 = (k1 + np.uint64(W1)) & _MASK
    return x0, x1, x2, x3


def seed_key(seed):
    """Key words from a 64-bit seed: (low 32 bits, high 32 bits)."""
    seed = int(seed)
    if seed < 0 or seed >= 1 << 64:
        raise ValueError("seed must fit in 64 unsigned bits")
    return seed & 0xFFFFFFFF, seed >> 32
