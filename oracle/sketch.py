"""Sketch matrices S drawn from the counter-based stream (oracle side).

The method samples an independent copy of S at every iteration (Alg. 3 and
Alg. 4, "sample an independent copy"); the experiments of Sec. 10 use two
distributions: S with i.i.d. standard normal entries ("gauss") and S made of q
distinct coordinate vectors chosen uniformly at random ("cols").

Stream definition (shared by specification, not by code, with the GPU side):

  key     = (seed, 0)
  counter = (block, k, kind, 0)      k = iteration index, kind 1 = gauss, 2 = cols
  words   = Philox4x64-10(counter, key)  -> four uint64 per block

Gaussian entry e = j*n + i of the n x q matrix (column-major) uses block e>>2,
word w = e&3.  Words (0,1) and (2,3) of a block form Box-Muller pairs
(Box & Muller 1958): u = ((x >> 11) + 0.5) * 2^-53, r = sqrt(-2 ln u_a),
t = 2*pi*u_b, z = r cos t for the even word and r sin t for the odd one.  z is
rounded once, to nearest-even, to 8 significant bits (a bfloat16 value) so
that S is an exact operand for any precision; the scale of S does not matter
(S G^-1 S^T is invariant under S -> cS).

Coordinate sketch for iteration k: Floyd's algorithm (Bentley & Floyd, CACM
1987, "A sample of brilliance") draws q distinct indices of [0, n): for
j = n-q .. n-1, t = uniform integer in [0, j]; insert t, or j if t is already in
the set.  Uniform integers use Lemire's multiply-and-reject method (ACM TOMS
2019, "Fast random integer generation in an interval") on the word stream
W[4b + w] = word w of block b.  The indices are returned sorted ascending
(S G^-1 S^T does not depend on the column order).
"""
import math

import numpy as np

from .philox import philox4x64

KIND_GAUSS = 1
KIND_COLS = 2

_TWO_PI = 2.0 * math.pi
_TWO_M53 = 2.0 ** -53


def stream_block(seed, k, kind, block):
    """Four uint64 words of the given block(s) of the iteration-k stream."""
    block = np.asarray(block, dtype=np.uint64)
    return philox4x64(block, np.uint64(k), np.uint64(kind), np.uint64(0),
                      np.uint64(seed), np.uint64(0))


def round_bf16(x):
    """Round float64 values to nearest-even with 8 significant bits.

    Works on the IEEE-754 bit pattern: 45 of the 52 stored mantissa bits are
    dropped with round-half-to-even.  Valid for finite normal inputs (sketch
    entries are always in that range).
    """
    x = np.asarray(x, dtype=np.float64)
    bits = x.view(np.uint64)
    drop = np.uint64(45)
    half_minus_one = np.uint64((1 << 44) - 1)
    lsb = (bits >> drop) & np.uint64(1)
    with np.errstate(over="ignore"):
        rounded = (bits + half_minus_one + lsb) & ~np.uint64((1 << 45) - 1)
    return rounded.view(np.float64)


def uniform53(words):
    """Map uint64 words to doubles in (0, 1): ((x >> 11) + 0.5) * 2^-53."""
    w = np.asarray(words, dtype=np.uint64)
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * _TWO_M53


def gaussian_sketch(seed, k, n, q):
    """n x q Gaussian sketch of iteration k (float64 array holding bf16 values)."""
    total = n * q
    nblocks = (total + 3) // 4
    w0, w1, w2, w3 = stream_block(seed, k, KIND_GAUSS, np.arange(nblocks))
    z = np.empty((nblocks, 4), dtype=np.float64)
    for col, (ua, ub) in enumerate(((w0, w1), (w2, w3))):
        r = np.sqrt(-2.0 * np.log(uniform53(ua)))
        t = _TWO_PI * uniform53(ub)
        z[:, 2 * col] = r * np.cos(t)
        z[:, 2 * col + 1] = r * np.sin(t)
    flat = round_bf16(z.reshape(-1)[:total])
    # entry e = j*n + i  ->  column-major n x q
    return flat.reshape(q, n).T.copy()


class _WordStream:
    """Sequential reader of the uint64 words of one iteration's stream."""

    def __init__(self, seed, k, kind):
        self.seed, self.k, self.kind = seed, k, kind
        self.pos = 0
        self._block = -1
        self._words = None

    def next(self):
        b, w = divmod(self.pos, 4)
        if b != self._block:
            self._words = [int(v) for v in stream_block(self.seed, self.k, self.kind, b)]
            self._block = b
        self.pos += 1
        return self._words[w]


def bounded(stream, m):
    """Uniform integer in [0, m) from the word stream (Lemire's method)."""
    x = stream.next()
    prod = x * m
    lo = prod & ((1 << 64) - 1)
    if lo < m:
        thresh = ((1 << 64) - m) % m
        while lo < thresh:
            x = stream.next()
            prod = x * m
            lo = prod & ((1 << 64) - 1)
    return prod >> 64


def coord_sketch(seed, k, n, q):
    """Sorted array of q distinct indices of [0, n) for iteration k (Floyd)."""
    if not (1 <= q <= n):
        raise ValueError("need 1 <= q <= n")
    stream = _WordStream(seed, k, KIND_COLS)
    chosen = set()
    for j in range(n - q, n):
        t = bounded(stream, j + 1)
        chosen.add(j if t in chosen else t)
    return np.array(sorted(chosen), dtype=np.int64)


def coord_matrix(idx, n):
    """The n x q matrix I[:, idx] whose columns are coordinate vectors."""
    S = np.zeros((n, len(idx)), dtype=np.float64)
    S[np.asarray(idx), np.arange(len(idx))] = 1.0
    return S


def sketch(seed, k, n, q, kind):
    """Dense float64 sketch of iteration k: 'gauss' or 'cols'."""
    if kind == "gauss":
        return gaussian_sketch(seed, k, n, q)
    if kind == "cols":
        return coord_matrix(coord_sketch(seed, k, n, q), n)
    raise ValueError(kind)
