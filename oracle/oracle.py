"""ctypes front end of the CPU oracle (``ck_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the GPU library.  It shares no code
with the library; it only marshals numpy arrays into the oracle's C calls.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ck_oracle.cpp")
LIB = os.path.join(HERE, "libck_oracle.so")

RANDOM_WALK, BFS, SORTED, QUEUE, RATTLE, HYBRID = range(6)
SCHEMES = {"random_walk": RANDOM_WALK, "bfs": BFS, "sorted": SORTED, "queue": QUEUE,
           "rattle": RATTLE, "hybrid": HYBRID}
ST_NOT_FOUND, ST_OK, ST_FAIL, ST_ABORTED, ST_BAD_KEY, ST_UPDATED, ST_STASHED = range(7)
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
BANDS = 200

_STAT_SCALARS = ["inserts_ok", "inserts_failed", "inserts_aborted", "inserts_bad_key",
                 "views", "views_all", "kicks", "max_kicks", "retries", "rounds",
                 "twin_updates", "lookups", "lookup_hits", "lookup_probes", "deletes",
                 "deletes_found", "delete_probes", "delete_retries", "stored",
                 "inserts_stashed"]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in _STAT_SCALARS] + [
        ("band_inserts", ctypes.c_uint64 * BANDS), ("band_views", ctypes.c_uint64 * BANDS),
        ("band_kicks", ctypes.c_uint64 * BANDS), ("band_fails", ctypes.c_uint64 * BANDS)]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain C++17, -O2)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
        L.ck_oracle_create.restype = vp
        L.ck_oracle_create.argtypes = [u64, i32, i32, i32, i32, i32, u32, u32, u32, u32, u64, u64]
        L.ck_oracle_destroy.argtypes = [vp]
        L.ck_oracle_hash.argtypes = [vp, u64, vp]
        L.ck_oracle_insert.argtypes = [vp, vp, vp, u64, vp, vp, vp, vp]
        L.ck_oracle_insert_ids.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp]
        L.ck_oracle_lookup.argtypes = [vp, vp, u64, vp, vp]
        L.ck_oracle_delete.argtypes = [vp, vp, u64, vp, vp]
        L.ck_oracle_overwrite.argtypes = [vp, vp, vp, u64, vp, vp]
        L.ck_oracle_upsert.argtypes = [vp, vp, vp, u64, vp, vp, vp, vp]
        L.ck_oracle_upsert_ids.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp]
        L.ck_oracle_export.argtypes = [vp, vp, vp, vp, vp]
        L.ck_oracle_set_stash.argtypes = [vp, ctypes.c_uint32]
        L.ck_oracle_set_hash_bias.argtypes = [vp, ctypes.c_uint32]
        L.ck_oracle_set_hash_bias.restype = ctypes.c_int
        L.ck_oracle_set_stash.restype = ctypes.c_int
        L.ck_oracle_export_stash.argtypes = [vp, vp, vp]
        L.ck_oracle_import_stash.argtypes = [vp, vp, vp]
        L.ck_oracle_import.argtypes = [vp, vp, vp, vp, vp]
        L.ck_oracle_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.ck_oracle_txn.argtypes = [vp, vp, vp, vp, vp, u64, vp, vp, vp, vp]
        L.ck_oracle_txn.restype = i32
        L.ck_oracle_set_txn_bins.argtypes = [vp, u32]
        L.ck_oracle_set_txn_bins.restype = i32
        L.ck_oracle_set_spawn_k.argtypes = [vp, u32]
        L.ck_oracle_set_spawn_k.restype = i32
        L.ck_oracle_log_spawns.argtypes = [vp, i32]
        L.ck_oracle_spawn_log.argtypes = [vp, vp, vp, u64]
        L.ck_oracle_spawn_log.restype = u64
        L.ck_oracle_insert_count.restype = u64
        L.ck_oracle_insert_count.argtypes = [vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleTable:
    """One cuckoo table of the oracle.  ``batch_ops`` is the sub-batch size of
    the phased-round protocol; ``batch_ops=1`` is the plain serial algorithm."""

    def __init__(self, bins, slots_per_bin=4, d=2, scheme="random_walk", ghost=False,
                 load_balance=False, max_chain=500, max_search=500, max_rounds=0,
                 batch_ops=1, hash_seed=0, rng_seed=0, stash=0, hash_bias=0, spawn_k=0):
        self.n, self.B, self.H = int(bins), int(slots_per_bin), int(d)
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        self._t = lib().ck_oracle_create(self.n, self.B, self.H, self.scheme, int(ghost),
                                         int(load_balance), max_chain, max_search,
                                         max_rounds, batch_ops, hash_seed, rng_seed)
        if not self._t:
            raise ValueError("oracle rejected the table parameters")
        self.stash = int(stash)
        if self.stash and lib().ck_oracle_set_stash(self._t, self.stash) != 0:
            raise ValueError("oracle rejected the stash size")
        self.hash_bias = int(hash_bias)
        if self.hash_bias and lib().ck_oracle_set_hash_bias(self._t, self.hash_bias) != 0:
            raise ValueError("oracle rejected the hash bias")
        # BFS / sorted search spawning k records at a time (0: one at a time)
        self.spawn_k = int(spawn_k)
        if self.spawn_k and lib().ck_oracle_set_spawn_k(self._t, self.spawn_k) != 0:
            raise ValueError("oracle rejected spawn_k")

    def __del__(self):
        if getattr(self, "_t", None):
            lib().ck_oracle_destroy(self._t)
            self._t = None

    def hash(self, key) -> list[int]:
        out = np.zeros(4, dtype=np.uint64)
        lib().ck_oracle_hash(self._t, int(key), _p(out))
        return [int(v) for v in out[: self.H]]

    def insert(self, keys, vals, op_ids=None):
        """Insert; ``op_ids`` optionally fixes each op's index for the walk's
        random choices (default: the table's running insert count)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        n = keys.size
        status = np.zeros(n, np.uint8)
        views = np.zeros(n, np.uint32)
        kicks = np.zeros(n, np.uint32)
        retries = np.zeros(n, np.uint32)
        if op_ids is None:
            lib().ck_oracle_insert(self._t, _p(keys), _p(vals), n, _p(status), _p(views),
                                   _p(kicks), _p(retries))
        else:
            ids = np.ascontiguousarray(op_ids, dtype=np.uint64)
            lib().ck_oracle_insert_ids(self._t, _p(keys), _p(vals), _p(ids), n, _p(status),
                                       _p(views), _p(kicks), _p(retries))
        return {"status": status, "views": views, "kicks": kicks, "retries": retries}

    def lookup(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.zeros(keys.size, np.uint64)
        found = np.zeros(keys.size, np.uint8)
        lib().ck_oracle_lookup(self._t, _p(keys), keys.size, _p(vals), _p(found))
        return vals, found

    def delete(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        found = np.zeros(keys.size, np.uint8)
        retries = np.zeros(keys.size, np.uint32)
        lib().ck_oracle_delete(self._t, _p(keys), keys.size, _p(found), _p(retries))
        return found, retries

    def upsert(self, keys, vals, op_ids=None):
        """Insert, or give a stored key its new value (status ST_UPDATED);
        ``op_ids`` as for insert."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        n = keys.size
        status = np.zeros(n, np.uint8)
        views = np.zeros(n, np.uint32)
        kicks = np.zeros(n, np.uint32)
        retries = np.zeros(n, np.uint32)
        if op_ids is None:
            lib().ck_oracle_upsert(self._t, _p(keys), _p(vals), n, _p(status), _p(views),
                                   _p(kicks), _p(retries))
        else:
            ids = np.ascontiguousarray(op_ids, dtype=np.uint64)
            lib().ck_oracle_upsert_ids(self._t, _p(keys), _p(vals), _p(ids), n, _p(status),
                                       _p(views), _p(kicks), _p(retries))
        return {"status": status, "views": views, "kicks": kicks, "retries": retries}

    def overwrite(self, keys, vals):
        """New values for stored keys; returns (status per op, rounds lost)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        found = np.zeros(keys.size, np.uint8)
        retries = np.zeros(keys.size, np.uint32)
        lib().ck_oracle_overwrite(self._t, _p(keys), _p(vals), keys.size, _p(found), _p(retries))
        return found, retries

    def export(self):
        S = self.n * self.B
        keys = np.zeros(S, np.uint64)
        vals = np.zeros(S, np.uint64)
        rattle = np.zeros(S, np.uint16)
        meta = np.zeros(self.n, np.uint32)
        lib().ck_oracle_export(self._t, _p(keys), _p(vals), _p(rattle), _p(meta))
        img = {"keys": keys, "vals": vals, "rattle": rattle, "meta": meta}
        if self.stash:
            sk = np.zeros(self.stash, np.uint64)
            sv = np.zeros(self.stash, np.uint64)
            lib().ck_oracle_export_stash(self._t, _p(sk), _p(sv))
            img["stash_keys"], img["stash_vals"] = sk, sv
        return img

    def load(self, img):
        lib().ck_oracle_import(self._t, _p(np.ascontiguousarray(img["keys"], np.uint64)),
                               _p(np.ascontiguousarray(img["vals"], np.uint64)),
                               _p(np.ascontiguousarray(img["rattle"], np.uint16)),
                               _p(np.ascontiguousarray(img["meta"], np.uint32)))
        if self.stash:
            lib().ck_oracle_import_stash(
                self._t, _p(np.ascontiguousarray(img["stash_keys"], np.uint64)),
                _p(np.ascontiguousarray(img["stash_vals"], np.uint64)))

    def stats(self) -> dict:
        s = _Stats()
        lib().ck_oracle_stats(self._t, ctypes.byref(s))
        out = {n: int(getattr(s, n)) for n in _STAT_SCALARS}
        for f in ("band_inserts", "band_views", "band_kicks", "band_fails"):
            out[f] = np.array(list(getattr(s, f)), dtype=np.uint64)
        return out

    def set_txn_bins(self, bins):
        """Bound on the distinct bins a transaction's plan may touch (default
        512, as the GPU library); a larger plan aborts."""
        if lib().ck_oracle_set_txn_bins(self._t, int(bins)) != 0:
            raise ValueError("bad bound")

    def transactions(self, kinds, keys, vals, txn_off):
        """Transactional batch (Sec. 8): transaction t is ops
        [txn_off[t], txn_off[t+1]) (kinds 0 lookup, 1 insert, 2 delete, 3
        overwrite).  Returns per-op status and value, and per-transaction
        commit round and lost rounds."""
        kinds = np.ascontiguousarray(kinds, dtype=np.uint8)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(vals, dtype=np.uint64)
        off = np.ascontiguousarray(txn_off, dtype=np.uint64)
        nt = off.size - 1
        status = np.zeros(keys.size, np.uint8)
        vout = np.zeros(keys.size, np.uint64)
        rnd = np.zeros(nt, np.uint32)
        ret = np.zeros(nt, np.uint32)
        if lib().ck_oracle_txn(self._t, _p(kinds), _p(keys), _p(vals), _p(off), nt, _p(status),
                               _p(vout), _p(rnd), _p(ret)) != 0:
            raise ValueError("transactions need a table without ghosts or a stash")
        return {"status": status, "value": vout, "round": rnd, "retries": ret}

    def log_spawns(self, on=True):
        """Start (clearing it) or stop the record of spawn-count increments."""
        lib().ck_oracle_log_spawns(self._t, int(bool(on)))

    def spawn_log(self):
        """(insert op index, bin) of every spawn-count increment recorded, in
        the order applied."""
        cnt = int(lib().ck_oracle_spawn_log(self._t, None, None, 0))
        ops, bins = np.zeros(cnt, np.uint64), np.zeros(cnt, np.uint64)
        lib().ck_oracle_spawn_log(self._t, _p(ops), _p(bins), cnt)
        return ops, bins

    @property
    def insert_count(self) -> int:
        return int(lib().ck_oracle_insert_count(self._t))
