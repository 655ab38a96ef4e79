"""Independent checks on canonical table images (keys, vals, rattle, meta).

Written from the definitions, not from either implementation: a vectorised
numpy multiply-shift hash, and the structural invariants every cuckoo table
must satisfy (Sec. 1: a stored key sits in one of its bins; Sec. 4: a
duplicate is a marked pair in the key's two bins with equal values)."""
from __future__ import annotations

import numpy as np

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
GOLDEN = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def hash_params(hash_seed: int, H: int = 4):
    s = hash_seed
    a, c = [], []
    for _ in range(H):
        s = (s + GOLDEN) & MASK
        a.append(_mix(s) | 1)
        s = (s + GOLDEN) & MASK
        c.append(_mix(s))
    return a, c


def _mulhi(z: np.ndarray, n: int) -> np.ndarray:
    assert n < (1 << 32)
    nn = np.uint64(n)
    hi = z >> np.uint64(32)
    lo = z & np.uint64(0xFFFFFFFF)
    return (hi * nn + ((lo * nn) >> np.uint64(32))) >> np.uint64(32)


def bins_of(keys: np.ndarray, n: int, H: int, hash_seed: int) -> np.ndarray:
    """(len(keys), H) bin indices: floor(((a_i x + c_i) mod 2^64) n / 2^64),
    stepped forward past earlier choices so the H bins are distinct."""
    a, c = hash_params(hash_seed, H)
    keys = np.asarray(keys, dtype=np.uint64)
    out = np.zeros((keys.size, H), dtype=np.uint64)
    with np.errstate(over="ignore"):
        for i in range(H):
            h = _mulhi(np.uint64(a[i]) * keys + np.uint64(c[i]), n)
            while True:
                clash = np.zeros(keys.size, bool)
                for j in range(i):
                    clash |= out[:, j] == h
                if not clash.any():
                    break
                h = np.where(clash, (h + np.uint64(1)) % np.uint64(n), h)
            out[:, i] = h
    return out


def check_invariants(img, n, B, H, hash_seed, ghost=False, rattle=False):
    """P1 placement, P2 uniqueness / ghost pairs.  Returns the stored key set."""
    keys, vals, meta = img["keys"], img["vals"], img["meta"]
    S = n * B
    assert keys.size == S and meta.size == n
    occ = keys != EMPTY
    slot_bin = np.repeat(np.arange(n, dtype=np.uint64), B)
    slot_idx = np.tile(np.arange(B), n)
    dupbit = ((meta[slot_bin.astype(np.int64)] >> slot_idx.astype(np.uint32)) & 1).astype(bool)
    assert not np.any(dupbit & ~occ), "duplicate mark on an empty slot"
    k = keys[occ]
    b = slot_bin[occ]
    hb = bins_of(k, n, H, hash_seed)
    assert np.all((hb == b[:, None]).any(axis=1)), "a key sits outside its bins"
    d = dupbit[occ]
    uk, counts = np.unique(k, return_counts=True)
    if not ghost:
        assert not d.any(), "duplicate marks without ghost insertions"
    cnt = dict(zip(uk.tolist(), counts.tolist()))
    # non-duplicates appear once; duplicates exactly twice, both marked, in
    # the key's two different bins, with equal values
    nd = k[~d]
    assert all(cnt[x] == 1 for x in nd.tolist()), "unmarked key stored twice"
    if d.any():
        dk = k[d]
        db = b[d]
        dv = vals[occ][d]
        order = np.argsort(dk, kind="stable")
        dk, db, dv = dk[order], db[order], dv[order]
        assert dk.size % 2 == 0
        assert np.all(dk[0::2] == dk[1::2]), "a duplicate without its twin"
        assert np.all(db[0::2] != db[1::2]), "ghost twins in the same bin"
        assert np.all(dv[0::2] == dv[1::2]), "ghost twins with different values"
        assert all(cnt[x] == 2 for x in dk[0::2].tolist())
    if rattle:
        r = img["rattle"][occ].astype(np.int64)
        assert np.all(r >= 1), "stored key with no try recorded"
        where = hb[np.arange(k.size), (r - 1) % H]
        assert np.all(where == b), "rattle counter does not name the key's bin"
    return set(uk.tolist())
