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


def _mix_np(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _mulhi(z: np.ndarray, n: int) -> np.ndarray:
    assert n < (1 << 32)
    nn = np.uint64(n)
    hi = z >> np.uint64(32)
    lo = z & np.uint64(0xFFFFFFFF)
    return (hi * nn + ((lo * nn) >> np.uint64(32))) >> np.uint64(32)


def bins_of(keys: np.ndarray, n: int, H: int, hash_seed: int, hash_bias: int = 0) -> np.ndarray:
    """(len(keys), H) bin indices: floor(((a_i x + c_i) mod 2^64) n / 2^64),
    stepped forward past earlier choices so the H bins are distinct.  With a
    bias level k, the lesser of that and the bin of w = mix64(a_i x + c_i)
    when the two low bits of w are below k."""
    a, c = hash_params(hash_seed, H)
    keys = np.asarray(keys, dtype=np.uint64)
    out = np.zeros((keys.size, H), dtype=np.uint64)
    with np.errstate(over="ignore"):
        for i in range(H):
            z = np.uint64(a[i]) * keys + np.uint64(c[i])
            h = _mulhi(z, n)
            if hash_bias:
                w = _mix_np(z)
                h = np.where((w & np.uint64(3)) < np.uint64(hash_bias), np.minimum(h, _mulhi(w, n)), h)
            while True:
                clash = np.zeros(keys.size, bool)
                for j in range(i):
                    clash |= out[:, j] == h
                if not clash.any():
                    break
                h = np.where(clash, (h + np.uint64(1)) % np.uint64(n), h)
            out[:, i] = h
    return out


def check_invariants(img, n, B, H, hash_seed, ghost=False, rattle=False, hash_bias=0):
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
    hb = bins_of(k, n, H, hash_seed, hash_bias)
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
    held = set(uk.tolist())
    if "stash_keys" in img:  # stashed keys: distinct, and in no bin
        sk = img["stash_keys"][img["stash_keys"] != EMPTY]
        assert np.unique(sk).size == sk.size, "a key stashed twice"
        assert not held.intersection(sk.tolist()), "a stashed key also sits in a bin"
        held.update(sk.tolist())
    return held


# ---------------------------------------------------------------------------
# the same checks in torch (wrapping int64 arithmetic), for full-size images
# on the GPU; held equal to the numpy checks above by a CPU test
# ---------------------------------------------------------------------------
def _i64(c: int) -> int:
    return c - (1 << 64) if c >= (1 << 63) else c


def bins_of_torch(keys, n: int, H: int, hash_seed: int):
    """bins_of() for an int64 tensor of uint64 bit patterns: (len, H) int64."""
    import torch
    assert n < (1 << 32)
    a, c = hash_params(hash_seed, H)
    m32 = 0xFFFFFFFF
    out = []
    for i in range(H):
        z = keys * _i64(a[i]) + _i64(c[i])
        hi = (z >> 32) & m32
        lo = z & m32
        h = ((hi * n + (((lo * n) >> 32) & m32)) >> 32) & m32
        while True:
            clash = torch.zeros_like(h, dtype=torch.bool)
            for j in range(i):
                clash |= out[j] == h
            if not bool(clash.any()):
                break
            h = torch.where(clash, (h + 1) % n, h)
        out.append(h)
    return torch.stack(out, dim=1)


def check_image_torch(img, n, B, H, hash_seed, ghost=False, rattle=False, device="cuda"):
    """check_invariants() on `device`.  Returns the number of distinct stored keys."""
    import torch
    keys = torch.from_numpy(np.ascontiguousarray(img["keys"]).view(np.int64)).to(device)
    vals = torch.from_numpy(np.ascontiguousarray(img["vals"]).view(np.int64)).to(device)
    meta = torch.from_numpy(np.ascontiguousarray(img["meta"]).astype(np.int64)).to(device)
    S = n * B
    assert keys.numel() == S and meta.numel() == n
    occ = keys != -1
    slot = torch.arange(S, device=device)
    sbin = slot // B
    dup = ((meta[sbin] >> (slot % B)) & 1).bool()
    assert not bool((dup & ~occ).any()), "duplicate mark on an empty slot"
    k, b, d, v = keys[occ], sbin[occ], dup[occ], vals[occ]
    del slot, sbin, dup
    hb = bins_of_torch(k, n, H, hash_seed)
    assert bool((hb == b[:, None]).any(dim=1).all()), "a key sits outside its bins"
    if not ghost:
        assert not bool(d.any()), "duplicate marks without ghost insertions"
    if rattle:
        r = torch.from_numpy(np.ascontiguousarray(img["rattle"]).astype(np.int64)).to(device)[occ]
        assert bool((r >= 1).all()), "stored key with no try recorded"
        where = hb[torch.arange(k.numel(), device=device), (r - 1) % H]
        assert bool((where == b).all()), "rattle counter does not name the key's bin"
    del hb
    ks, order = torch.sort(k, stable=True)
    uk, counts = torch.unique_consecutive(ks, return_counts=True)
    cnt = torch.repeat_interleave(counts, counts)
    ds = d[order]
    assert bool((cnt[~ds] == 1).all()), "unmarked key stored twice"
    if bool(ds.any()):
        assert bool((cnt[ds] == 2).all()), "a duplicate without its twin"
        bs, vs = b[order][ds], v[order][ds]
        assert bool((ks[ds][0::2] == ks[ds][1::2]).all()), "a duplicate without its twin"
        assert bool((bs[0::2] != bs[1::2]).all()), "ghost twins in the same bin"
        assert bool((vs[0::2] == vs[1::2]).all()), "ghost twins with different values"
    return int(uk.numel())
