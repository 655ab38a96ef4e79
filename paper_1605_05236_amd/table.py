"""ctypes binding of libck (include/ck.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libck.so``.  PyTorch provides device memory (table storage, key/value and
result tensors) and the HIP stream.  If the library has not been built the
binding raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libck.so")

SCHEMES = {"random_walk": 0, "bfs": 1, "sorted": 2, "queue": 3, "rattle": 4, "hybrid": 5}
OP_NOT_FOUND, OP_OK, OP_FAIL_CHAIN, OP_ABORTED, OP_BAD_KEY, OP_UPDATED, OP_STASHED = range(7)
BANDS = 200
EMPTY_KEY = 0xFFFFFFFFFFFFFFFF

_SCALARS = ["inserts_ok", "inserts_failed", "inserts_aborted", "inserts_bad_key", "views",
            "views_all", "kicks", "max_kicks", "retries", "rounds", "twin_updates", "lookups",
            "lookup_hits", "lookup_probes", "deletes", "deletes_found", "delete_probes",
            "delete_retries", "stored"]


class CkOptions(ctypes.Structure):
    _fields_ = [("ghost", ctypes.c_uint32), ("load_balance", ctypes.c_uint32),
                ("max_chain", ctypes.c_uint32), ("max_search", ctypes.c_uint32),
                ("max_rounds", ctypes.c_uint32), ("batch_ops", ctypes.c_uint32),
                ("hash_seed", ctypes.c_uint64), ("rng_seed", ctypes.c_uint64),
                ("evict_wgs_per_cu", ctypes.c_uint32), ("enqueue_rounds", ctypes.c_uint32),
                ("stash", ctypes.c_uint32), ("hash_bias", ctypes.c_uint32),
                ("spawn_k", ctypes.c_uint32)]


class CkStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in _SCALARS] + [
        ("band_inserts", ctypes.c_uint64 * BANDS), ("band_views", ctypes.c_uint64 * BANDS),
        ("band_kicks", ctypes.c_uint64 * BANDS), ("band_fails", ctypes.c_uint64 * BANDS),
        ("arena_moves", ctypes.c_uint64), ("inserts_stashed", ctypes.c_uint64)]


class CkKernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("ms", ctypes.c_double)]


_TIMED = ["plan_fresh", "plan_evict", "plan_delete", "commit", "stats", "lookup"]
TIME_ALL = 63


def time_mask(classes) -> int:
    """Bit mask of kernel classes for timing(enable=...)."""
    if classes is True:
        return TIME_ALL
    if not classes:
        return 0
    return sum(1 << _TIMED.index(c) for c in classes)


class CkTiming(ctypes.Structure):
    _fields_ = [(n, CkKernelTime) for n in _TIMED] + [("evict_views", ctypes.c_uint64)]


class CkError(RuntimeError):
    pass


_lib = None

EXPORTED = ["ck_default_options", "ck_storage_bytes", "ck_create", "ck_clear", "ck_insert", "ck_insert_ex",
            "ck_lookup", "ck_lookup_lpp", "ck_delete", "ck_delete_noalloc", "ck_overwrite",
            "ck_upsert", "ck_transact",
            "ck_stats_get", "ck_stats_reset", "ck_export_stash", "ck_import_stash",
            "ck_group_export_stash",
            "ck_export", "ck_import", "ck_hash", "ck_insert_count", "ck_destroy", "ck_strerror",
            "ck_timing_enable", "ck_timing_get", "ck_group_storage_bytes", "ck_group_create",
            "ck_group_insert", "ck_group_lookup", "ck_group_delete", "ck_group_overwrite",
            "ck_group_upsert", "ck_group_export_table",
            "ck_group_stats_get", "ck_group_timing_enable", "ck_group_timing_get",
            "ck_group_clear", "ck_group_insert_count", "ck_group_destroy"]


def load_library(path: str = LIB_PATH):
    """Open libck.so and declare its signatures (no GPU call is made)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise CkError(f"{path} is missing: build it with __graft_entry__.build() "
                      "(hipcc, gfx950); there is no CPU fallback")
    L = ctypes.CDLL(path)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.ck_default_options.argtypes = [ctypes.POINTER(CkOptions)]
    L.ck_default_options.restype = None
    L.ck_storage_bytes.argtypes = [u64, u32, u32, ctypes.POINTER(ctypes.c_size_t)]
    L.ck_create.argtypes = [u64, u32, u32, i32, ctypes.POINTER(CkOptions), vp, ctypes.c_size_t,
                            vp, ctypes.POINTER(vp)]
    L.ck_clear.argtypes = [vp, vp]
    L.ck_insert.argtypes = [vp, vp, vp, u64, vp, vp]
    L.ck_insert_ex.argtypes = [vp, vp, vp, u64, vp, vp, vp, vp, vp]
    L.ck_lookup.argtypes = [vp, vp, u64, vp, vp, vp]
    L.ck_lookup_lpp.argtypes = [vp, vp, u64, vp, vp, u32, vp]
    L.ck_delete.argtypes = [vp, vp, u64, vp, vp]
    L.ck_delete_noalloc.argtypes = [vp, vp, u64, vp, vp]
    L.ck_transact.argtypes = [vp, vp, vp, vp, vp, u32, vp, vp, vp, vp]
    L.ck_overwrite.argtypes = [vp, vp, vp, u64, vp, vp]
    L.ck_upsert.argtypes = [vp, vp, vp, u64, vp, vp, vp, vp, vp]
    L.ck_export_stash.argtypes = [vp, vp, vp, vp]
    L.ck_import_stash.argtypes = [vp, vp, vp, vp]
    L.ck_group_export_stash.argtypes = [vp, u32, vp, vp, vp]
    L.ck_stats_get.argtypes = [vp, ctypes.POINTER(CkStats), vp]
    L.ck_stats_reset.argtypes = [vp, vp]
    L.ck_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ck_import.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ck_hash.argtypes = [vp, u64, vp]
    L.ck_insert_count.argtypes = [vp]
    L.ck_insert_count.restype = u64
    L.ck_destroy.argtypes = [vp]
    L.ck_timing_enable.argtypes = [vp, u32]
    L.ck_timing_get.argtypes = [vp, ctypes.POINTER(CkTiming), vp]
    L.ck_group_storage_bytes.argtypes = [u32, vp, u32, u32, ctypes.POINTER(ctypes.c_size_t)]
    L.ck_group_create.argtypes = [u32, vp, u32, u32, i32, ctypes.POINTER(CkOptions), vp,
                                  ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ck_group_insert.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp, vp]
    L.ck_group_lookup.argtypes = [vp, vp, vp, u64, vp, vp, u32, vp]
    L.ck_group_delete.argtypes = [vp, vp, vp, u64, vp, vp]
    L.ck_group_overwrite.argtypes = [vp, vp, vp, vp, u64, vp, vp]
    L.ck_group_upsert.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp, vp]
    L.ck_group_export_table.argtypes = [vp, u32, vp, vp, vp, vp, vp]
    L.ck_group_stats_get.argtypes = [vp, ctypes.POINTER(CkStats), vp]
    L.ck_group_timing_enable.argtypes = [vp, u32]
    L.ck_group_timing_get.argtypes = [vp, ctypes.POINTER(CkTiming), vp]
    L.ck_group_clear.argtypes = [vp, vp]
    L.ck_group_insert_count.argtypes = [vp]
    L.ck_group_insert_count.restype = u64
    L.ck_group_destroy.argtypes = [vp]
    L.ck_strerror.argtypes = [i32]
    L.ck_strerror.restype = ctypes.c_char_p
    for f in ("ck_storage_bytes", "ck_create", "ck_clear", "ck_insert", "ck_insert_ex", "ck_lookup",
              "ck_lookup_lpp", "ck_delete", "ck_delete_noalloc", "ck_transact", "ck_overwrite", "ck_upsert", "ck_stats_get",
              "ck_stats_reset", "ck_export", "ck_export_stash", "ck_import_stash",
              "ck_group_export_stash",
              "ck_import", "ck_hash", "ck_destroy", "ck_timing_enable", "ck_timing_get",
              "ck_group_storage_bytes", "ck_group_create", "ck_group_insert", "ck_group_lookup",
              "ck_group_delete", "ck_group_overwrite", "ck_group_upsert",
              "ck_group_export_table", "ck_group_stats_get",
              "ck_group_timing_enable", "ck_group_timing_get", "ck_group_clear",
              "ck_group_destroy"):
        getattr(L, f).restype = i32
    if path == LIB_PATH:
        _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise CkError(f"libck error {rc}: {load_library().ck_strerror(rc).decode()}")


def _ptr(t) -> int:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def as_device_keys(keys, device="cuda"):
    """uint64 numpy keys -> int64 device tensor holding the same bits."""
    import torch
    if isinstance(keys, torch.Tensor):
        return keys.to(device=device, dtype=torch.int64).contiguous()
    a = np.ascontiguousarray(keys, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(a).to(device)


def storage_bytes(bins: int, slots_per_bin: int = 4, d: int = 2) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().ck_storage_bytes(bins, slots_per_bin, d, ctypes.byref(out)))
    return int(out.value)


class CuckooTable:
    """One device-resident cuckoo table.  Storage is a torch uint8 tensor that
    the table keeps alive; ``stream=None`` uses torch's current stream."""

    def __init__(self, bins, slots_per_bin=4, d=2, scheme="random_walk", ghost=False,
                 load_balance=False, max_chain=500, max_search=500, max_rounds=0,
                 batch_ops=1 << 20, hash_seed=0, rng_seed=0, device="cuda", stream=None,
                 evict_wgs_per_cu=0, enqueue_rounds=0, stash=0, hash_bias=0, spawn_k=0):
        import torch
        L = load_library()
        self.n, self.B, self.H = int(bins), int(slots_per_bin), int(d)
        self.stash = int(stash)
        self.device = torch.device(device)
        self.value_dtype = torch.int32 if self.B == 1 else torch.int64
        opt = CkOptions()
        L.ck_default_options(ctypes.byref(opt))
        opt.ghost, opt.load_balance = int(ghost), int(load_balance)
        opt.max_chain, opt.max_search, opt.max_rounds = max_chain, max_search, max_rounds
        opt.batch_ops, opt.hash_seed, opt.rng_seed = batch_ops, hash_seed, rng_seed
        opt.evict_wgs_per_cu, opt.enqueue_rounds = evict_wgs_per_cu, enqueue_rounds
        opt.stash, opt.hash_bias = self.stash, int(hash_bias)
        opt.spawn_k = int(spawn_k)
        self.storage = torch.empty(storage_bytes(self.n, self.B, self.H), dtype=torch.uint8,
                                   device=self.device)
        h = ctypes.c_void_p()
        sch = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        _check(L.ck_create(self.n, self.B, self.H, sch, ctypes.byref(opt), _ptr(self.storage),
                           self.storage.numel(), _stream(stream), ctypes.byref(h)))
        self._h = h
        self._L = L

    def close(self):
        if getattr(self, "_h", None):
            self._L.ck_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None):
        """Empty the table and zero its counters (storage is kept)."""
        _check(self._L.ck_clear(self._h, _stream(stream)))

    # ---- batched operations (device tensors in, device tensors out)
    def insert(self, keys, vals, stream=None, diagnostics=True):
        import torch
        n = keys.numel()
        status = torch.empty(n, dtype=torch.uint8, device=self.device)
        if not diagnostics:
            _check(self._L.ck_insert(self._h, _ptr(keys), _ptr(vals), n, _ptr(status),
                                     _stream(stream)))
            return {"status": status}
        views = torch.empty(n, dtype=torch.int32, device=self.device)
        kicks = torch.empty_like(views)
        retries = torch.empty_like(views)
        _check(self._L.ck_insert_ex(self._h, _ptr(keys), _ptr(vals), n, _ptr(status),
                                    _ptr(views), _ptr(kicks), _ptr(retries), _stream(stream)))
        return {"status": status, "views": views, "kicks": kicks, "retries": retries}

    def lookup(self, keys, lanes_per_probe=0, stream=None, out=None, found=None):
        import torch
        n = keys.numel()
        if out is None:
            out = torch.empty(n, dtype=self.value_dtype, device=self.device)
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(self._L.ck_lookup_lpp(self._h, _ptr(keys), n, _ptr(out), _ptr(found),
                                     lanes_per_probe, _stream(stream)))
        return out, found

    def delete(self, keys, stream=None):
        import torch
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=self.device)
        _check(self._L.ck_delete(self._h, _ptr(keys), keys.numel(), _ptr(found),
                                 _stream(stream)))
        return found

    def delete_noalloc(self, keys, stream=None):
        """As delete, with the round scratch taken from the library's fixed
        per-device array (ck_delete_noalloc): no device allocation."""
        import torch
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=self.device)
        _check(self._L.ck_delete_noalloc(self._h, _ptr(keys), keys.numel(), _ptr(found),
                                         _stream(stream)))
        return found

    def transact(self, kinds, keys, vals, txn_off, stream=None):
        """Transactional batch (ck_transact, Sec. 8): uint8 kinds (0 lookup,
        1 insert, 2 delete, 3 overwrite), int64 keys and values, int32
        transaction offsets (n_txn + 1) on the device.  Returns per-op status
        and value, and per-transaction commit round."""
        import torch
        n = keys.numel()
        nt = txn_off.numel() - 1
        status = torch.empty(n, dtype=torch.uint8, device=self.device)
        vout = torch.empty(n, dtype=torch.int64, device=self.device)
        rnd = torch.empty(max(nt, 1), dtype=torch.int32, device=self.device)
        _check(self._L.ck_transact(self._h, _ptr(kinds), _ptr(keys), _ptr(vals), _ptr(txn_off),
                                   nt, _ptr(status), _ptr(vout), _ptr(rnd), _stream(stream)))
        return {"status": status, "value": vout, "round": rnd[:nt]}

    def overwrite(self, keys, vals, stream=None):
        """New values for stored keys (absent keys are reported, not inserted)."""
        import torch
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=self.device)
        _check(self._L.ck_overwrite(self._h, _ptr(keys), _ptr(vals), keys.numel(), _ptr(found),
                                    _stream(stream)))
        return found

    def upsert(self, keys, vals, stream=None, diagnostics=True):
        """Insert absent keys; stored keys get the new value (status UPDATED)."""
        import torch
        n = keys.numel()
        status = torch.empty(n, dtype=torch.uint8, device=self.device)
        if diagnostics:
            views = torch.empty(n, dtype=torch.int32, device=self.device)
            kicks, retries = torch.empty_like(views), torch.empty_like(views)
            ptrs = (_ptr(views), _ptr(kicks), _ptr(retries))
        else:
            ptrs = (None, None, None)
        _check(self._L.ck_upsert(self._h, _ptr(keys), _ptr(vals), n, _ptr(status), *ptrs,
                                 _stream(stream)))
        if not diagnostics:
            return {"status": status}
        return {"status": status, "views": views, "kicks": kicks, "retries": retries}

    # ---- host-side views
    def stats(self, stream=None) -> dict:
        s = CkStats()
        _check(self._L.ck_stats_get(self._h, ctypes.byref(s), _stream(stream)))
        out = {n: int(getattr(s, n)) for n in _SCALARS}
        for f in ("band_inserts", "band_views", "band_kicks", "band_fails"):
            out[f] = np.array(list(getattr(s, f)), dtype=np.uint64)
        out["arena_moves"] = int(s.arena_moves)
        out["inserts_stashed"] = int(s.inserts_stashed)
        return out

    def reset_stats(self, stream=None):
        _check(self._L.ck_stats_reset(self._h, _stream(stream)))

    def export(self, stream=None) -> dict:
        S = self.n * self.B
        keys = np.zeros(S, np.uint64)
        vals = np.zeros(S, np.uint64)
        rattle = np.zeros(S, np.uint16)
        meta = np.zeros(self.n, np.uint32)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(self._L.ck_export(self._h, c(keys), c(vals), c(rattle), c(meta), _stream(stream)))
        img = {"keys": keys, "vals": vals, "rattle": rattle, "meta": meta}
        if self.stash:
            sk, sv = np.zeros(self.stash, np.uint64), np.zeros(self.stash, np.uint64)
            _check(self._L.ck_export_stash(self._h, c(sk), c(sv), _stream(stream)))
            img["stash_keys"], img["stash_vals"] = sk, sv
        return img

    def load(self, img, stream=None):
        c = lambda a: np.ascontiguousarray(a).ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        arrs = [np.ascontiguousarray(img["keys"], np.uint64),
                np.ascontiguousarray(img["vals"], np.uint64),
                np.ascontiguousarray(img["rattle"], np.uint16),
                np.ascontiguousarray(img["meta"], np.uint32)]
        _check(self._L.ck_import(self._h, *[c(a) for a in arrs], _stream(stream)))
        if self.stash:
            _check(self._L.ck_import_stash(
                self._h, c(np.ascontiguousarray(img["stash_keys"], np.uint64)),
                c(np.ascontiguousarray(img["stash_vals"], np.uint64)), _stream(stream)))

    def timing(self, enable=None, stream=None):
        """Enable per-kernel event timing (True = every class, or a list of
        class names; False or [] disables; enabling resets it), or read it."""
        if enable is not None:
            _check(self._L.ck_timing_enable(self._h, time_mask(enable)))
            return None
        t = CkTiming()
        _check(self._L.ck_timing_get(self._h, ctypes.byref(t), _stream(stream)))
        out = {n: {"launches": int(getattr(t, n).launches), "ms": float(getattr(t, n).ms)}
               for n in _TIMED}
        out["evict_views"] = int(t.evict_views)
        return out

    def hash(self, key) -> list[int]:
        out = np.zeros(4, np.uint64)
        _check(self._L.ck_hash(self._h, int(key), out.ctypes.data_as(ctypes.c_void_p)))
        return [int(v) for v in out[: self.H]]

    @property
    def insert_count(self) -> int:
        return int(self._L.ck_insert_count(self._h))


def _options(ghost, load_balance, max_chain, max_search, max_rounds, batch_ops, hash_seed,
             rng_seed, evict_wgs_per_cu=0, enqueue_rounds=0, stash=0, hash_bias=0, spawn_k=0):
    opt = CkOptions()
    load_library().ck_default_options(ctypes.byref(opt))
    opt.ghost, opt.load_balance = int(ghost), int(load_balance)
    opt.max_chain, opt.max_search, opt.max_rounds = max_chain, max_search, max_rounds
    opt.batch_ops, opt.hash_seed, opt.rng_seed = batch_ops, hash_seed, rng_seed
    opt.evict_wgs_per_cu, opt.enqueue_rounds = evict_wgs_per_cu, enqueue_rounds
    opt.stash, opt.hash_bias = stash, hash_bias
    opt.spawn_k = spawn_k
    return opt


def _timing_dict(t: CkTiming) -> dict:
    out = {n: {"launches": int(getattr(t, n).launches), "ms": float(getattr(t, n).ms)}
           for n in _TIMED}
    out["evict_views"] = int(t.evict_views)
    return out


class CuckooGroup:
    """Many independent tables of uneven sizes in one device allocation, served
    by the same launches: every op carries its table index (int32 tensor)."""

    def __init__(self, bins, slots_per_bin=4, d=2, scheme="queue", ghost=False,
                 load_balance=False, max_chain=500, max_search=500, max_rounds=0,
                 batch_ops=1 << 20, hash_seed=0, rng_seed=0, device="cuda", stream=None,
                 evict_wgs_per_cu=0, enqueue_rounds=0, stash=0, hash_bias=0, spawn_k=0):
        import torch
        L = load_library()
        self.stash = int(stash)
        self.bins = np.ascontiguousarray(bins, dtype=np.uint64)
        self.n_tables, self.B, self.H = int(self.bins.size), int(slots_per_bin), int(d)
        self.device = torch.device(device)
        self.value_dtype = torch.int32 if self.B == 1 else torch.int64
        size = ctypes.c_size_t()
        _check(L.ck_group_storage_bytes(self.n_tables, self.bins.ctypes.data_as(ctypes.c_void_p),
                                        self.B, self.H, ctypes.byref(size)))
        self.storage = torch.empty(int(size.value), dtype=torch.uint8, device=self.device)
        opt = _options(ghost, load_balance, max_chain, max_search, max_rounds, batch_ops,
                       hash_seed, rng_seed, evict_wgs_per_cu, enqueue_rounds, self.stash,
                       int(hash_bias), int(spawn_k))
        h = ctypes.c_void_p()
        sch = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        _check(L.ck_group_create(self.n_tables, self.bins.ctypes.data_as(ctypes.c_void_p),
                                 self.B, self.H, sch, ctypes.byref(opt), _ptr(self.storage),
                                 self.storage.numel(), _stream(stream), ctypes.byref(h)))
        self._h = h
        self._L = L

    def close(self):
        if getattr(self, "_h", None):
            self._L.ck_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None):
        _check(self._L.ck_group_clear(self._h, _stream(stream)))

    def insert(self, tables, keys, vals, stream=None, diagnostics=True):
        import torch
        n = keys.numel()
        status = torch.empty(n, dtype=torch.uint8, device=self.device)
        if diagnostics:
            views = torch.empty(n, dtype=torch.int32, device=self.device)
            kicks, retries = torch.empty_like(views), torch.empty_like(views)
            ptrs = (_ptr(views), _ptr(kicks), _ptr(retries))
        else:
            ptrs = (None, None, None)
        _check(self._L.ck_group_insert(self._h, _ptr(tables), _ptr(keys), _ptr(vals), n,
                                       _ptr(status), *ptrs, _stream(stream)))
        if not diagnostics:
            return {"status": status}
        return {"status": status, "views": views, "kicks": kicks, "retries": retries}

    def lookup(self, tables, keys, lanes_per_probe=0, stream=None, out=None, found=None):
        import torch
        n = keys.numel()
        if out is None:
            out = torch.empty(n, dtype=self.value_dtype, device=self.device)
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(self._L.ck_group_lookup(self._h, _ptr(tables), _ptr(keys), n, _ptr(out),
                                       _ptr(found), lanes_per_probe, _stream(stream)))
        return out, found

    def delete(self, tables, keys, stream=None):
        import torch
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=self.device)
        _check(self._L.ck_group_delete(self._h, _ptr(tables), _ptr(keys), keys.numel(),
                                       _ptr(found), _stream(stream)))
        return found

    def overwrite(self, tables, keys, vals, stream=None):
        import torch
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=self.device)
        _check(self._L.ck_group_overwrite(self._h, _ptr(tables), _ptr(keys), _ptr(vals),
                                          keys.numel(), _ptr(found), _stream(stream)))
        return found

    def upsert(self, tables, keys, vals, stream=None, diagnostics=True):
        import torch
        n = keys.numel()
        status = torch.empty(n, dtype=torch.uint8, device=self.device)
        if diagnostics:
            views = torch.empty(n, dtype=torch.int32, device=self.device)
            kicks, retries = torch.empty_like(views), torch.empty_like(views)
            ptrs = (_ptr(views), _ptr(kicks), _ptr(retries))
        else:
            ptrs = (None, None, None)
        _check(self._L.ck_group_upsert(self._h, _ptr(tables), _ptr(keys), _ptr(vals), n,
                                       _ptr(status), *ptrs, _stream(stream)))
        if not diagnostics:
            return {"status": status}
        return {"status": status, "views": views, "kicks": kicks, "retries": retries}

    def export_table(self, table, stream=None) -> dict:
        nb = int(self.bins[table])
        S = nb * self.B
        keys = np.zeros(S, np.uint64)
        vals = np.zeros(S, np.uint64)
        rattle = np.zeros(S, np.uint16)
        meta = np.zeros(nb, np.uint32)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(self._L.ck_group_export_table(self._h, int(table), c(keys), c(vals), c(rattle),
                                             c(meta), _stream(stream)))
        img = {"keys": keys, "vals": vals, "rattle": rattle, "meta": meta}
        if self.stash:
            sk, sv = np.zeros(self.stash, np.uint64), np.zeros(self.stash, np.uint64)
            _check(self._L.ck_group_export_stash(self._h, int(table), c(sk), c(sv),
                                                 _stream(stream)))
            img["stash_keys"], img["stash_vals"] = sk, sv
        return img

    def stats(self, stream=None) -> dict:
        st = CkStats()
        _check(self._L.ck_group_stats_get(self._h, ctypes.byref(st), _stream(stream)))
        out = {n: int(getattr(st, n)) for n in _SCALARS}
        out["inserts_stashed"] = int(st.inserts_stashed)
        return out

    def timing(self, enable=None, stream=None):
        if enable is not None:
            _check(self._L.ck_group_timing_enable(self._h, time_mask(enable)))
            return None
        t = CkTiming()
        _check(self._L.ck_group_timing_get(self._h, ctypes.byref(t), _stream(stream)))
        return _timing_dict(t)

    @property
    def insert_count(self) -> int:
        return int(self._L.ck_group_insert_count(self._h))
