"""Plan cache on the CPU: the checksummed per-pair butterfly records that sht_plan_ex reads
and writes with opts.cache_dir, exercised through the host-only entry points
(sht_plan_cache_append / _check / _read) on butterflies the host builder makes from the
oracle's dense Q^{(m,p)}.  Round trip bit for bit, a flipped byte in a record or in the header,
a torn last record, resumption in pair order, and the argument checks."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_0910_5435_amd import Butterfly, _lib, plan_cache_append, plan_cache_check

L, C, EPS = 8, 4, 1e-13
NP = 4 * L


def _depth(l, C, mp):
    n0 = (2 * l - mp // 2 + 1) // 2
    return max(0, math.ceil(math.log2(math.ceil(n0 / C)))) if n0 > C else 0


def _butterfly(mp):
    q = oracle.dense_q(L, mp // 2, mp % 2)
    return Butterfly(q, leaf_width=C, eps=EPS, levels=_depth(L, C, mp))


def _path(d):
    bits = np.array([EPS]).view(np.uint64)[0]
    return os.path.join(str(d), f"sht_plan_l{L}_C{C}_e{bits:016x}_v1.cache")


def _write(d, upto=NP):
    bfs = [_butterfly(mp) for mp in range(upto)]
    for mp, bf in enumerate(bfs):
        plan_cache_append(d, L, EPS, C, mp, bf)
    return bfs


def _record_offsets(path):
    """Start offsets of every record (after the 36-byte header), and the file size."""
    data = open(path, "rb").read()
    offs, off = [], 36
    while off < len(data):
        offs.append(off)
        size = int.from_bytes(data[off + 4:off + 12], "little")
        off += 4 + 8 + size + 4
    return offs, len(data)


def _same_tree(a, b):
    assert (a.levels, a.k_max, a.factor_entries, a.m_max_words) == (b.levels, b.k_max, b.factor_entries,
                                                                     b.m_max_words)
    for t in range(a.levels + 1):
        for r in range(1 << t):
            for c in range(1 << (a.levels - t)):
                sa, ra, Ta = a.block(t, r, c)
                sb, rb, Tb = b.block(t, r, c)
                assert np.array_equal(sa, sb) and np.array_equal(ra, rb) and np.array_equal(Ta, Tb)
    for r in range(1 << a.levels):
        ra, Sa, ca = a.final(r)
        rb, Sb, cb = b.final(r)
        assert ra == rb and np.array_equal(Sa, Sb) and np.array_equal(ca, cb)


def test_round_trip_every_pair(tmp_path):
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_EINVAL, 0)  # no file yet
    bfs = _write(tmp_path)
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_OK, NP)
    for mp, bf in enumerate(bfs):
        _same_tree(bf, Butterfly.from_plan_cache(tmp_path, L, EPS, C, mp))


def test_flipped_byte_in_a_record_is_corrupt(tmp_path):
    _write(tmp_path)
    path = _path(tmp_path)
    offs, _ = _record_offsets(path)
    j = 11
    data = bytearray(open(path, "rb").read())
    data[offs[j] + 20] ^= 0x10  # inside record j's payload
    open(path, "wb").write(bytes(data))
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_ECORRUPT, j)
    with pytest.raises(_lib.ShtError) as ei:
        Butterfly.from_plan_cache(tmp_path, L, EPS, C, j)
    assert ei.value.status == _lib.SHT_ECORRUPT
    Butterfly.from_plan_cache(tmp_path, L, EPS, C, j - 1)  # the prefix before it is intact
    # appending is refused until the file is rebuilt
    with pytest.raises(_lib.ShtError) as ei:
        plan_cache_append(tmp_path, L, EPS, C, j, _butterfly(j))
    assert ei.value.status == _lib.SHT_ECORRUPT


def test_flipped_byte_in_the_header_is_corrupt(tmp_path):
    _write(tmp_path, upto=3)
    path = _path(tmp_path)
    data = bytearray(open(path, "rb").read())
    data[26] ^= 0x01  # inside the stored eps
    open(path, "wb").write(bytes(data))
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_ECORRUPT, 0)


def test_torn_record_and_resume_in_pair_order(tmp_path):
    bfs = _write(tmp_path, upto=9)
    path = _path(tmp_path)
    offs, size = _record_offsets(path)
    # a crash while the last record was written: its tail is missing
    with open(path, "r+b") as f:
        f.truncate(size - 7)
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_ECORRUPT, 8)
    # cut at a record boundary: an intact, incomplete cache that resumes at pair 5
    with open(path, "r+b") as f:
        f.truncate(offs[5])
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_OK, 5)
    with pytest.raises(_lib.ShtError) as ei:  # records go in pair order
        plan_cache_append(tmp_path, L, EPS, C, 6, bfs[6])
    assert ei.value.status == _lib.SHT_EINVAL
    for mp in range(5, NP):
        plan_cache_append(tmp_path, L, EPS, C, mp, bfs[mp] if mp < len(bfs) else _butterfly(mp))
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_OK, NP)
    _same_tree(bfs[7], Butterfly.from_plan_cache(tmp_path, L, EPS, C, 7))


def test_trailing_bytes_after_the_last_record_are_corrupt(tmp_path):
    _write(tmp_path)
    with open(_path(tmp_path), "ab") as f:
        f.write(b"\x00" * 5)
    assert plan_cache_check(tmp_path, L, EPS, C) == (_lib.SHT_ECORRUPT, NP)


def test_append_checks_the_pair_shape(tmp_path):
    bf = _butterfly(1)  # pair 1's shape offered as pair 0
    with pytest.raises(_lib.ShtError) as ei:
        plan_cache_append(tmp_path, L, EPS, C, 0, Butterfly(oracle.dense_q(L, 3, 0), leaf_width=C, eps=EPS,
                                                            levels=_depth(L, C, 6)))
    assert ei.value.status == _lib.SHT_EINVAL
    with pytest.raises(_lib.ShtError) as ei:
        plan_cache_append(tmp_path, L, EPS, C, 4 * L, bf)
    assert ei.value.status == _lib.SHT_EINVAL
    # another eps or leaf width names another file
    _write(tmp_path, upto=2)
    assert plan_cache_check(tmp_path, L, 1e-12, C)[0] == _lib.SHT_EINVAL
    assert plan_cache_check(tmp_path, L, EPS, 2 * C)[0] == _lib.SHT_EINVAL
