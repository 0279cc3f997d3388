"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

Both the oracle and the HIP path draw every random number of the sampler from
this published generator, so that a GPU run can be replayed draw for draw.
Specification shared by both sides:

* key = (seed, stream), counter = (c0, c1, c2, c3), 64-bit words.
* ten rounds of
      (hi0, lo0) = mulhilo(0xD2E7470EE14C6C93, x0)
      (hi1, lo1) = mulhilo(0xCA5A826395121157, x2)
      x = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
  with the key bumped by (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B) between
  rounds.
* uniform from a 64-bit word w: U = (w >> 11) * 2^-53, in [0, 1).
* the q-th draw of a sequence (c1, c2, c3) is word (q mod 4) of the block at
  counter (q div 4, c1, c2, c3).

Streams: 0 = nested-sampling draws, c1 = walker, c2 = step, c3 = iteration;
1 = shrinkage replicates of the evidence error, c1 = replicate.

Pinned by: numpy.random.Philox (an independent implementation of the same
published generator).
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """(hi, lo) 64-bit halves of the 128-bit product of uint64 arrays."""
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Ten-round Philox4x64 block for arrays of counters (broadcast)."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for r in range(10):
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + W0
            k1 = k1 + W1
    return x0, x1, x2, x3


def to_unit(w):
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniforms(seed, stream, c1, c2, c3, draws):
    """Uniforms U[..., q] for draw indices ``draws`` of the sequences (c1, c2, c3).

    c1, c2, c3 broadcast together to a shape S; the result has shape S + (len(draws),).
    """
    draws = np.asarray(draws, dtype=np.uint64)
    c1, c2, c3 = np.broadcast_arrays(np.asarray(c1, dtype=np.uint64),
                                     np.asarray(c2, dtype=np.uint64),
                                     np.asarray(c3, dtype=np.uint64))
    shape = c1.shape
    blk = (draws >> np.uint64(2))
    lane = (draws & np.uint64(3)).astype(np.int64)
    ex = (Ellipsis,) + (None,)
    w = philox4x64(blk[(None,) * len(shape)], c1[ex], c2[ex], c3[ex],
                   np.uint64(seed), np.uint64(stream))
    words = np.stack(w, axis=-1)                                  # S + (n, 4)
    picked = np.take_along_axis(words, np.broadcast_to(lane, shape + lane.shape)[..., None], axis=-1)[..., 0]
    return to_unit(picked)


def normals(U_even, U_odd):
    """Box-Muller (cosine branch): sqrt(-2 ln(1 - U1)) cos(2 pi U2)."""
    return np.sqrt(-2.0 * np.log1p(-U_even)) * np.cos(2.0 * np.pi * U_odd)
