"""Pins of the wavelet codec oracle (oracle/codec.py).

* lifting by hand on one line: [1, 4, 2, 8] -> [2.25, 4.125, 2.5, 6];
* perfect reconstruction of the transform (no quantisation) to rounding;
* a constant cube transforms to its value in the one coarsest coefficient and zeros elsewhere;
  a field linear along an axis has zero details except at the symmetric extension;
* zigzag map by hand, a packed group by hand, and pack/unpack round trips;
* the reconstruction error after quantisation stays within gain * step / 2 cell by cell, gain
  being the synthesis operator's row-sum norm computed by brute force;
* the whole stream: header fields, offsets, and a decompress(compress()) round trip.
"""
import struct

import numpy as np
import pytest

from oracle import codec as C


def test_lifting_by_hand():
    y = C._fwd_lines(np.array([1.0, 4.0, 2.0, 8.0]))
    assert np.array_equal(y, [2.25, 4.125, 2.5, 6.0])
    assert np.array_equal(C._inv_lines(y), [1.0, 4.0, 2.0, 8.0])


@pytest.mark.parametrize("n", [4, 8, 16])
def test_perfect_reconstruction(n):
    x = np.random.default_rng(n).standard_normal((n, n, n))
    L = C.levels_for(n)
    assert np.abs(C.idwt3(C.dwt3(x, L), L) - x).max() <= 1e-14


@pytest.mark.parametrize("n", [4, 16])
def test_constant_and_linear_fields(n):
    L = C.levels_for(n)
    c = C.dwt3(np.full((n, n, n), 2.5), L)
    assert c[0, 0, 0] == 2.5 and np.count_nonzero(c) == 1
    i = np.arange(n, dtype=np.float64)
    lin = np.broadcast_to(0.25 * i[None, None, :] - 1.0, (n, n, n))   # exact arithmetic
    y = C._fwd_lines(lin)
    d = y[..., n // 2:]
    assert np.abs(d[..., :-1]).max() == 0.0 and np.abs(d[..., -1]).min() > 0


def test_zigzag_and_a_packed_group_by_hand():
    assert list(C.zigzag([0, -1, 1, -2, 2])) == [0, 1, 2, 3, 4]
    assert list(C.unzigzag([0, 1, 2, 3, 4])) == [0, -1, 1, -2, 2]
    q = np.zeros(64, dtype=np.int64)
    q[1] = -2                      # zigzag 3: width 2, value 3 at bits 2..3 -> word 12
    q[33] = 1                      # second group: zigzag 2, width 2, at bits 2..3 -> word 8
    buf = C.pack_cube(q)
    assert buf == bytes([2, 2, 0, 0]) + struct.pack("<4I", 12, 0, 8, 0)
    back, used = C.unpack_cube(buf, 64)
    assert used == len(buf) and np.array_equal(back, q)


def test_pack_round_trip_all_widths():
    rng = np.random.default_rng(3)
    q = np.concatenate([rng.integers(-(1 << b), 1 << b, 32) for b in range(0, 31)] +
                       [np.zeros(32, dtype=np.int64)])
    q = np.concatenate([q, np.zeros((-q.size) % 512, dtype=np.int64)])
    back, used = C.unpack_cube(C.pack_cube(q), q.size)
    assert np.array_equal(back, q)


@pytest.mark.parametrize("n", [4, 8])
def test_error_within_the_synthesis_bound(n):
    g = C.synthesis_gain(n)
    rng = np.random.default_rng(7)
    nc = 5
    x = rng.standard_normal(nc * n ** 3)
    step = 1e-3
    y = C.decompress(C.compress(x, n, nc, step))
    err = np.abs(y - x).max()
    assert err <= g * step / 2 * (1 + 1e-12)
    assert err >= 0.05 * step       # quantisation really happened


def test_stream_header_and_round_trip():
    n, nc = 8, 3
    rng = np.random.default_rng(9)
    x = np.cumsum(rng.standard_normal(nc * n ** 3)) * 1e-2     # correlated values
    s = C.compress(x, n, nc, 1e-4)
    assert s[:4] == b"BCMW"
    ver, ncub, nn, L, zero, step = struct.unpack_from("<IIIIId", s, 4)
    assert (ver, ncub, nn, L, zero, step) == (1, nc, n, 3, 0, 1e-4)
    offs = np.frombuffer(s, dtype="<u8", count=nc + 1, offset=32)
    assert offs[0] == 0 and len(s) == 32 + 8 * (nc + 1) + int(offs[-1])
    assert np.all(np.diff(offs.astype(np.int64)) > 0)
    y = C.decompress(s)
    assert np.abs(y - x).max() <= C.synthesis_gain(n) * 1e-4 / 2
