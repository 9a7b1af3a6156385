"""Counter-based Gaussian noise: Philox4x32-10 and the Box-Muller transform.

Large segments (tens of GB) are generated on the device by the library's
noise kernel; this module is the host-side definition of the same values, so
that any element of such a segment can be regenerated on the host from its
index alone.  Both follow the published definitions:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key; each
  of 10 rounds multiplies counter words 0 and 2 by the constants 0xD2511F53
  and 0xCD9E8D57, mixes the high halves of the products with words 1 and 3
  and the key, and the key is bumped by the Weyl constants 0x9E3779B9 and
  0xBB67AE85 between rounds.
* Box-Muller (Box and Muller 1958): two uniforms u1, u2 in (0, 1) give the
  independent normals sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).

Stream layout (the contract the device generator follows):
  complex element e = ((t * nbl + b) * nchan + c) * npol + p, t the absolute
  integration index; Philox block n = e // 2 with counter (n mod 2^32,
  n // 2^32, stream, 0) and key (seed mod 2^32, seed // 2^32).  Element e
  takes words (x0, x1) of its block when e is even, (x2, x3) when odd; with
  u_k = (x_k + 1/2) / 2^32 in float64, Re = r cos(theta), Im = r sin(theta),
  r = sqrt(-2 ln u_a), theta = 2 pi u_b, all in float64, then rounded to
  float32 (complex64).  FP16 storage is the round-to-nearest-even of those
  float32 values.
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
TWO_PI = 6.283185307179586  # float64 nearest to 2 pi
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10: uint32-valued arrays in, four uint32 arrays
    out."""
    c = [np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64)
    k1 = np.asarray(k1, dtype=np.uint64)
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & _MASK
        k1 = (k1 + np.uint64(W1)) & _MASK
    return [x.astype(np.uint32) for x in c]


def element_values(e, seed, stream=0):
    """complex64 noise values of the global element indices e (int64 array)."""
    e = np.asarray(e, dtype=np.int64)
    n = (e >> 1).astype(np.uint64)
    x = philox4x32_10(n & _MASK, n >> np.uint64(32), np.full(n.shape, stream, np.uint64),
                      np.zeros(n.shape, np.uint64), np.uint64(seed) & _MASK,
                      np.uint64(seed) >> np.uint64(32))
    odd = (e & 1).astype(bool)
    xa = np.where(odd, x[2], x[0]).astype(np.float64)
    xb = np.where(odd, x[3], x[1]).astype(np.float64)
    u1 = (xa + 0.5) / 4294967296.0
    u2 = (xb + 0.5) / 4294967296.0
    r = np.sqrt(-2.0 * np.log(u1))
    th = TWO_PI * u2
    out = np.empty(e.shape, dtype=np.complex64)
    out.real = (r * np.cos(th)).astype(np.float32)
    out.imag = (r * np.sin(th)).astype(np.float32)
    return out


def segment(seed, nint, nbl, nchan, npol, t_first=0, stream=0):
    """complex64 [nint][nbl][nchan][npol] noise of integrations
    t_first .. t_first + nint - 1."""
    per = nbl * nchan * npol
    e = np.arange(per * nint, dtype=np.int64) + np.int64(t_first) * per
    return element_values(e, seed, stream).reshape(nint, nbl, nchan, npol)


def gather(seed, nbl, nchan, npol, t, b, c, p, stream=0):
    """Noise values at broadcastable index arrays (t, b, c, p)."""
    t, b, c, p = np.broadcast_arrays(*(np.asarray(x, dtype=np.int64) for x in (t, b, c, p)))
    e = ((t * nbl + b) * nchan + c) * npol + p
    return element_values(e, seed, stream)
