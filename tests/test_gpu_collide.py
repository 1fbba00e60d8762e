"""Anchors whose out-neighbours all share one home bucket of the closure's
hash table: the keys fill a run of buckets, the inserts mark every bucket
they pass over, and each lookup of a key past its home bucket walks the
marked run.  Counts and splits must equal the oracle's, exact and sampled,
for an anchor of the wave-per-item kernel (d+ = 100) and one of the block
kernel (d+ = 300).

The bucket of a key is the top lg bits of a 32-bit multiplicative hash of its
id (the closure kernels' table layout, restated here only to pick colliding
ids); keys that agree in the top 10 bits share their home bucket for every
table size up to 1024 buckets."""
import sys

import numpy as np
import pytest

import oracle
import synth


def _home(w, lg):
    prod = ((w & 0xFFFFFF) * 0x9E3779 + (w >> 24)) & 0xFFFFFFFF
    return prod >> (32 - lg)


def _colliding(count, lo, hi):
    ids = np.arange(lo, hi, dtype=np.int64)
    top = _home(ids, 10)
    vals, cnt = np.unique(top, return_counts=True)
    best = vals[np.argmax(cnt)]
    pick = ids[top == best][:count]
    assert len(pick) == count, (count, cnt.max())
    return pick


def _graph(d, seed):
    """A sparse background (so that m' is large and the anchor stays light),
    anchor 0 joined to d colliding keys, the keys joined among themselves at
    random (the triangles through the anchor) and each key given filler
    edges into the background so that it outranks the anchor."""
    rng = np.random.default_rng(seed)
    nb = 400000
    base = 1000  # background vertices [base, base + nb)
    _, s0, d0 = synth.uniform_pairs(nb, 1500000, seed=seed)
    src = [s0.astype(np.int64) + base]
    dst = [d0.astype(np.int64) + base]
    keys = _colliding(d, base + nb, base + nb + 2000000)
    n = int(keys.max()) + 1
    src.append(np.zeros(d, np.int64))
    dst.append(keys)
    iu = np.triu_indices(d, 1)
    sel = rng.random(len(iu[0])) < 0.3
    src.append(keys[iu[0][sel]])
    dst.append(keys[iu[1][sel]])
    fill = d + 20  # more than the anchor's degree
    src.append(np.repeat(keys, fill))
    dst.append(rng.integers(base, base + nb, size=d * fill))
    return n, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)


GRAPHS = {"wave_d100": _graph(100, 1), "block_d300": _graph(300, 2)}


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_colliding_keys_match_oracle(gpu, name):
    n, s, d = GRAPHS[name]
    g = gpu.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    for p, seed in ((1.0, 0), (0.5, 1)):
        sys.stdout.write("collide %s p=%g\n" % (name, p))
        sys.stdout.flush()
        want = oracle.count_split(og if p == 1.0 else oracle.sample(og, p, seed), 1, 1)
        got = gpu.tc_count_exact(g) if p == 1.0 else gpu.tc_estimate(g, p, [seed])[0][0]
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert got[k] == want[k], (name, p, k, got[k], want[k])
    g.free()


def test_colliding_ids_share_a_bucket():
    keys = _colliding(300, 10 ** 6, 3 * 10 ** 6)
    for lg in (7, 8, 9, 10):
        assert len(set(_home(keys, lg).tolist())) == 1
