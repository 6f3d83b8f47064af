"""Per-cube lossy wavelet compression of a cell field (checkpoints): the paper's compression
algorithm (Sec. 6.4.1, Alg. "Compression algorithm"): a discrete wavelet transform of each cube
on its own, one level of quantisation, and an entropy coder, the cubes' streams concatenated
behind a header that records each cube's size.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Readings (the paper names the steps, not their parameters):
  w1  wavelet: the CDF 5/3 (LeGall) biorthogonal wavelet by lifting, separable along x, then y,
      then z, on levels of n, n/2, ... down to 2 cells per edge (n = 16: 16, 8, 4 and 2), with
      symmetric extension at the cube's faces; after each level the coarse half of each axis is
      stored first (in-place Mallat layout).  On one line x[0..m-1] (m even):
        d_i = x_{2i+1} - (x_{2i} + x_{2i+2}) / 2     (x_m read as x_{m-2})
        s_i = x_{2i} + (d_{i-1} + d_i) / 4            (d_{-1} read as d_0)
      and the line becomes s_0..s_{m/2-1}, d_0..d_{m/2-1}.  The inverse undoes the two lifting
      steps in the opposite order.
  w2  the transform covers the cube's cells only: the paper extends it to the halo so that a
      restarted rank can rebuild its ghost layers without an exchange; on one device the
      face buffers are re-exported from the decoded cubes, so the stream holds no halo.
  w3  quantisation: q = round-half-even(c / step) of every coefficient c, one uniform step for
      the whole field; reconstruction c' = q * step.
  w4  entropy coder (the paper uses zlib): adaptive bit packing.  The n^3 codes of a cube, in
      storage order, form groups of 32; each code is mapped to an unsigned integer by the
      zigzag map (q >= 0 -> 2q, q < 0 -> -2q - 1), and a group is stored as w = the bit length
      of its largest value (0..32), then its 32 values at w bits each, value j at bits
      j w .. j w + w - 1 of the group's w little-endian 32-bit words.
Stream layout (little-endian):
  bytes 0..3   magic b"BCMW"          4..7   version (1)
  8..11        number of cubes        12..15 n (cells per cube edge)
  16..19       levels                 20..23 zero
  24..31       step (FP64)
  32..         cube offsets, (number of cubes + 1) x u64, relative to the data start
  data         per cube: the G = n^3 / 32 group widths (one byte each, padded with zeros to a
               multiple of 4), then the groups' words in order.
The arithmetic of the transform is written with the operations in the order shown above and
no fused multiply-add, so that a GPU implementation doing the same IEEE operations produces
the same coefficients, codes and bytes.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"BCMW"
VERSION = 1


def levels_for(n):
    """Transform levels for n cells per edge: down to 2 cells (n = 16: 4 levels)."""
    return int(np.log2(n))


# -- 1-D lifting along the last axis of an array ------------------------------------------------
def _fwd_lines(x):
    m = x.shape[-1]
    ev = x[..., 0::2]
    od = x[..., 1::2]
    right = np.concatenate([ev[..., 1:], ev[..., -1:]], axis=-1)   # x_{2i+2}, x_m -> x_{m-2}
    d = od - (ev + right) / 2.0
    left = np.concatenate([d[..., :1], d[..., :-1]], axis=-1)      # d_{i-1}, d_{-1} -> d_0
    s = ev + (left + d) / 4.0
    return np.concatenate([s, d], axis=-1)


def _inv_lines(y):
    m = y.shape[-1]
    h = m // 2
    s = y[..., :h]
    d = y[..., h:]
    left = np.concatenate([d[..., :1], d[..., :-1]], axis=-1)
    ev = s - (left + d) / 4.0
    right = np.concatenate([ev[..., 1:], ev[..., -1:]], axis=-1)
    od = d + (ev + right) / 2.0
    x = np.empty_like(y)
    x[..., 0::2] = ev
    x[..., 1::2] = od
    return x


def dwt3(cube, levels):
    """Forward transform of cube [n, n, n] ([k][j][i]) in place, levels of w1."""
    c = np.array(cube, dtype=np.float64, copy=True)
    m = c.shape[0]
    for _ in range(levels):
        blk = c[:m, :m, :m]
        blk[...] = _fwd_lines(blk)                                   # along x (i)
        blk[...] = np.swapaxes(_fwd_lines(np.swapaxes(blk, 1, 2)), 1, 2)   # along y (j)
        blk[...] = np.swapaxes(_fwd_lines(np.swapaxes(blk, 0, 2)), 0, 2)   # along z (k)
        m //= 2
    return c


def idwt3(coef, levels):
    c = np.array(coef, dtype=np.float64, copy=True)
    n = c.shape[0]
    for L in reversed(range(levels)):
        m = n >> L
        blk = c[:m, :m, :m]
        blk[...] = np.swapaxes(_inv_lines(np.swapaxes(blk, 0, 2)), 0, 2)   # z first
        blk[...] = np.swapaxes(_inv_lines(np.swapaxes(blk, 1, 2)), 1, 2)   # then y
        blk[...] = _inv_lines(blk)                                   # then x
    return c


# -- quantisation and codes --------------------------------------------------------------------
def quantise(coef, step):
    q = np.rint(np.asarray(coef) / step)
    assert np.all(np.abs(q) < 2.0 ** 30), "step too small for the field (codes beyond 2^30)"
    return q.astype(np.int64)


def zigzag(q):
    q = np.asarray(q, dtype=np.int64)
    return np.where(q >= 0, 2 * q, -2 * q - 1).astype(np.uint64)


def unzigzag(z):
    z = np.asarray(z, dtype=np.int64)
    return np.where(z % 2 == 0, z // 2, -(z + 1) // 2)


def _bitlen(v):
    v = int(v)
    return v.bit_length()


def pack_cube(codes):
    """Bytes of one cube: group widths (padded to 4) then the packed groups (w4)."""
    z = zigzag(codes.ravel())
    G = z.size // 32
    widths = [max(_bitlen(v) for v in z[g * 32:(g + 1) * 32]) for g in range(G)]
    head = bytes(widths) + bytes((-G) % 4)
    words = []
    for g, w in enumerate(widths):
        acc = 0
        for j, v in enumerate(z[g * 32:(g + 1) * 32]):
            acc |= int(v) << (j * w)
        words += [(acc >> (32 * t)) & 0xFFFFFFFF for t in range(w)]
    return head + struct.pack(f"<{len(words)}I", *words)


def unpack_cube(buf, n3):
    G = n3 // 32
    widths = list(buf[:G])
    pos = G + (-G) % 4
    out = np.empty(n3, dtype=np.int64)
    for g, w in enumerate(widths):
        words = struct.unpack_from(f"<{w}I", buf, pos)
        pos += 4 * w
        acc = 0
        for t, wd in enumerate(words):
            acc |= wd << (32 * t)
        mask = (1 << w) - 1
        for j in range(32):
            out[g * 32 + j] = (acc >> (j * w)) & mask if w else 0
    return unzigzag(out), pos


def compress(field, n, n_cubes, step):
    """The whole stream (bytes) of a cube-major field."""
    L = levels_for(n)
    f = np.asarray(field, dtype=np.float64).reshape(n_cubes, n, n, n)
    parts = [pack_cube(quantise(dwt3(f[c], L), step)) for c in range(n_cubes)]
    offs = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.uint64)
    head = MAGIC + struct.pack("<IIIIId", VERSION, n_cubes, n, L, 0, step)
    return head + offs.astype("<u8").tobytes() + b"".join(parts)


def decompress(stream):
    assert stream[:4] == MAGIC
    version, n_cubes, n, L, _, step = struct.unpack_from("<IIIIId", stream, 4)
    assert version == VERSION
    offs = np.frombuffer(stream, dtype="<u8", count=n_cubes + 1, offset=32)
    data = 32 + 8 * (n_cubes + 1)
    out = np.empty((n_cubes, n, n, n))
    for c in range(n_cubes):
        q, used = unpack_cube(stream[data + int(offs[c]): data + int(offs[c + 1])], n ** 3)
        assert used == int(offs[c + 1] - offs[c])
        out[c] = idwt3((q * step).reshape(n, n, n), L)
    return out.reshape(-1)


def synthesis_gain(n):
    """Max over cells of sum_j |S_ij|, S = the inverse transform (coefficients -> cells): with
    every code off by at most 1/2, |x - x'| <= gain * step / 2 cell by cell."""
    L = levels_for(n)
    N = n ** 3
    S = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        S[:, j] = idwt3(e.reshape(n, n, n), L).ravel()
    return float(np.abs(S).sum(axis=1).max())
