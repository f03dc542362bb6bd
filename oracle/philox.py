"""Philox4x32-10 and Box-Muller Gaussian samples (oracle side, FP64).

Alg. 1 step 4 asks for a Gaussian matrix M with prod_{i!=n} I_i rows and K_n columns.  The
oracle and the GPU library draw the same entries because each implements, independently,
the same counter-based generator:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
  SC'11): 4x32-bit counter, 2x32-bit key, ten rounds.  One round multiplies counter words 0
  and 2 by the constants M0, M1 into 64-bit products (hi, lo), and forms the new counter
  (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).  Between rounds the key is bumped by the Weyl
  constants W0, W1.
* Box-Muller (Box & Muller 1958): two uniforms u_a, u_b in (0,1) give
  r cos(2 pi u_b), r sin(2 pi u_b) with r = sqrt(-2 ln u_a).

Stream layout (the contract shared with the GPU side):
  key     = (seed mod 2^32, seed >> 32)
  counter = (c mod 2^32, c >> 32, stream_word, tensor_id), c = call index
  element e of a stream comes from call c = e >> 2, lane e & 3; lanes 0,1 are the
  Box-Muller pair of words (w0, w1), lanes 2,3 the pair of words (w2, w3)
  uniform u(w) = (w + 1/2) 2^-32, so u is never 0 or 1
  stream_word = tag << 24 | mode << 16 | factor << 8 (mode, factor 0-based)

Parity: pinned by the published Philox known-answer vectors and by distribution tests.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

TAG_OMEGA = 1  # Gaussian test matrices of Alg. 1 step 4
TAG_KR = 3     # Gaussian factors of the Khatri-Rao structured test matrices

def stream_word(tag, mode, factor=0):
    """stream_word = tag << 24 | mode << 16 | factor << 8 (factor: the other mode whose
    Gaussian factor a Khatri-Rao test matrix draws; 0 otherwise)."""
    return ((tag & 0xFF) << 24) | ((mode & 0xFF) << 16) | ((factor & 0xFF) << 8)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ``ctr`` is four arrays (or ints) of 32-bit words,
    ``key`` two ints.  Returns four uint64 arrays holding 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in ctr)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = m0 * c0  # < 2^64: exact in uint64
        p1 = m1 * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0),
                          p1 & _MASK,
                          (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1),
                          p0 & _MASK)
    return c0, c1, c2, c3


def uniform(w):
    """u(w) = (w + 1/2) 2^-32 in FP64 (exact)."""
    return (np.asarray(w, dtype=np.float64) + 0.5) * 2.0 ** -32


def box_muller(wa, wb):
    """Pair of N(0,1) samples from two 32-bit words (Box & Muller 1958)."""
    r = np.sqrt(-2.0 * np.log(uniform(wa)))
    t = (2.0 * np.pi) * uniform(wb)
    return r * np.cos(t), r * np.sin(t)


def normals(seed, stream, tensor_id, start, count):
    """Elements [start, start+count) of the Gaussian stream (seed, stream, tensor_id), FP64."""
    count = int(count)
    if count <= 0:
        return np.zeros(0)
    start = int(start)
    first = start >> 2
    last = (start + count - 1) >> 2
    c = np.arange(first, last + 1, dtype=np.uint64)
    w0, w1, w2, w3 = philox4x32_10(
        (c & _MASK, c >> np.uint64(32), np.uint64(stream), np.uint64(tensor_id)),
        (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    z0, z1 = box_muller(w0, w1)
    z2, z3 = box_muller(w2, w3)
    z = np.stack([z0, z1, z2, z3], axis=1).reshape(-1)
    off = start - 4 * first
    return z[off:off + count]
