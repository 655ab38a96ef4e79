/*
 * ck.h -- C ABI of libck, batched cuckoo hash tables on AMD Instinct MI355X
 * (gfx950) with the kick-out eviction schemes of Kuszmaul, "Fast Concurrent
 * Cuckoo Kick-out Eviction Schemes for High-Density Tables" (arXiv 1605.05236).
 *
 * A table has `bins` bins of `slots_per_bin` slots and `d` hash functions
 * (Sec. 1: two bins per key, bins of 4 or 8 slots; Sec. 7: d-ary tables with
 * single-slot bins).  Keys are 64-bit; the all-ones key is reserved to mark an
 * empty slot.  Values are 64-bit for slots_per_bin >= 2 and 32-bit for
 * single-slot bins (whose slot also carries the 16-bit rattle counter of
 * Sec. 7).
 *
 * Concurrency model.  A batch of inserts (or deletes) is applied in phased
 * rounds: every pending op plans its kick-out chain against the same snapshot
 * of the table, claims every bin its plan writes (lowest op index wins a bin;
 * the per-bin claim word is the paper's claim flag, Sec. 8.2), and the ops that
 * own all their bins commit their chains in reverse order (the "system
 * transaction" order of Sec. 8.2).  The rest re-plan next round.  The result is
 * a pure function of the table, the batch and the seeds, independent of thread
 * timing; a batch of one op is the paper's serial algorithm.
 *
 * Conventions for every call:
 *   - returns ck_status (0 = CK_OK, negative = error); nothing else signals
 *     errors and no exception crosses the ABI;
 *   - `d_` pointers are device pointers (HIP global memory) owned by the
 *     caller; `h_` pointers are host pointers owned by the caller;
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it; ck_insert, ck_upsert, ck_delete and ck_overwrite wait once per
 *     sub-batch for its round counters (one sub-batch ahead), so they return
 *     with every round complete;
 *   - calls on one table must not overlap; tables are independent.
 */
#ifndef CK_H
#define CK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CK_EMPTY_KEY 0xFFFFFFFFFFFFFFFFull
#define CK_BANDS 200 /* density bands of 0.5 % */

typedef struct ck_table ck_table; /* opaque host-side handle */

typedef enum {
  CK_OK = 0,
  CK_EINVAL = -1,       /* bad argument (geometry, sizes, null pointers) */
  CK_ENOMEM = -2,       /* storage too small or scratch allocation failed */
  CK_EDEVICE = -3,      /* a HIP runtime call failed (sticky device error) */
  CK_EUNSUPPORTED = -5  /* valid request this library does not implement */
} ck_status;

/* Kick-out eviction schemes.
 *   CK_RANDOM_WALK  random kicking: a random victim in a random bin, the
 *                   victim moves to one of its other bins (Sec. 1, Sec. 6).
 *   CK_BFS          breadth-first search for the shortest chain (Sec. 1, 5).
 *   CK_SORTED       sorted search by per-bin spawn count (Sec. 5).
 *   CK_QUEUE        queue-kicking with hit counters, load and hit balancing
 *                   (Sec. 6); two hash functions only.
 *   CK_RATTLE       rattle-kicking, d-ary tables with single-slot bins (Sec. 7).
 *   CK_HYBRID       the sorted-search / BFS hybrid: records spawned by depth,
 *                   then by spawn count (Sec. 5). */
typedef enum {
  CK_RANDOM_WALK = 0,
  CK_BFS = 1,
  CK_SORTED = 2,
  CK_QUEUE = 3,
  CK_RATTLE = 4,
  CK_HYBRID = 5
} ck_scheme;

/* Per-op result bytes written to device arrays. */
enum {
  CK_OP_NOT_FOUND = 0, /* lookup/delete: key absent */
  CK_OP_OK = 1,        /* inserted / found / deleted */
  CK_OP_FAIL_CHAIN = 2,/* insert: chain or search cap exceeded; table unchanged */
  CK_OP_ABORTED = 3,   /* lost its claims in max_rounds rounds; table unchanged */
  CK_OP_BAD_KEY = 4,   /* the key is CK_EMPTY_KEY */
  CK_OP_UPDATED = 5,   /* upsert: the key was stored and got the new value */
  CK_OP_STASHED = 6    /* insert: the chain failed and the key went to the stash */
};

typedef struct {
  uint32_t ghost;        /* ghost insertions (Sec. 4); d == 2 only */
  uint32_t load_balance; /* fresh insert into the less full bin (Sec. 2);
                            CK_QUEUE always balances */
  uint32_t max_chain;    /* kicks (walk schemes) or tries (rattle) before an
                            insert fails; <= 2048 */
  uint32_t max_search;   /* bins viewed before a BFS/sorted insert fails; <= 1024 */
  uint32_t max_rounds;   /* lost rounds before CK_OP_ABORTED; 0 = never */
  uint32_t batch_ops;    /* sub-batch size of the round protocol; results
                            depend on it (1 = serial) */
  uint64_t hash_seed;    /* seeds the hash multipliers */
  uint64_t rng_seed;     /* seeds the random walk's choices */
  uint32_t evict_wgs_per_cu; /* kick-out planner workgroups per compute unit;
                                0 = as many as the LDS budget allows (<= 32).
                                Performance only: results do not depend on it */
  uint32_t enqueue_rounds;   /* rounds enqueued per sub-batch before the host
                                first looks at its counters (more follow in
                                groups of this size while ops are pending);
                                0 = as many as the larger of the last two
                                insert sub-batches took (deletes: one more than
                                the last), then groups of two.  Performance only */
  uint32_t stash;            /* stash entries per table (Sec. 2), <= 64; 0 = no
                                stash.  An insert whose chain fails puts its key
                                in the first free entry (CK_OP_STASHED); lookups,
                                deletes, overwrites and upserts search the stash
                                after the key's bins, as one more probe */
  uint32_t hash_bias;        /* 0: uniform hashes (Sec. 3).  1-4: biased hashes
                                (Sec. 9): for each choice, w = mix64(a_i x + c_i)
                                (mix64: splitmix64's output function) and, when
                                the two low bits of w are below hash_bias, the
                                bin is the lesser of the bins of a_i x + c_i and
                                of w, so low bins are favoured */
  uint32_t spawn_k;          /* 0 or 1: searches spawn one record at a time.
                                k >= 2 (CK_BFS and CK_SORTED, d == 2,
                                slots_per_bin 4 or 8, k <= 32 / slots_per_bin):
                                the search spawns the k records at the front of
                                its order together and views their candidate
                                bins at once (Sec. 5, Prefetching); the first
                                bin with room among them ends the chain.  Results
                                depend on k */
} ck_options;

/* Counters of one table since creation (or the last ck_stats_reset). */
typedef struct {
  uint64_t inserts_ok, inserts_failed, inserts_aborted, inserts_bad_key;
  uint64_t views;       /* bins viewed by the plans that decided each insert */
  uint64_t views_all;   /* bins viewed by every plan, including lost rounds */
  uint64_t kicks, max_kicks, retries, rounds, twin_updates;
  uint64_t lookups, lookup_hits, lookup_probes;
  uint64_t deletes, deletes_found, delete_probes, delete_retries;
  uint64_t stored;      /* distinct keys currently held, in bins or the stash */
  /* per 0.5 % density band: inserts, their bins viewed, kicks, failures;
     an op's density is the table's had its sub-batch been applied in op order */
  uint64_t band_inserts[CK_BANDS], band_views[CK_BANDS];
  uint64_t band_kicks[CK_BANDS], band_fails[CK_BANDS];
  uint64_t arena_moves; /* capacity of the plan arena (moves of one round's
                           kick-out plans); it doubles when a round runs out */
  uint64_t inserts_stashed; /* inserts whose chain failed and whose key went to
                               the stash (counted in band_fails and `stored`,
                               not in inserts_failed) */
} ck_stats;

/* Defaults: no ghosts, first fit, max_chain 500, max_search 500, max_rounds 0,
   batch_ops 2^20, hash_seed 0, rng_seed 0. */
void ck_default_options(ck_options* opt);

/* Device bytes a table of this geometry needs: n bins of B slots (Sec. 1;
   single-slot bins with d choices, Sec. 7), plus the per-bin metadata word
   (duplicate marks of Sec. 4, spawn count of Sec. 5, hit counter of Sec. 6)
   and the per-bin claim word (Sec. 8.2).  Pure host arithmetic, no device
   call.  Errors: CK_EINVAL for an unsupported geometry or a null `out`. */
ck_status ck_storage_bytes(uint64_t bins, uint32_t slots_per_bin, uint32_t d, size_t* out);

/* Create a table (Sec. 1: n bins of B slots, two hash functions; Sec. 7: d
   hash functions over single-slot bins; the scheme is one of the kick-out
   mechanisms of Secs. 1, 5, 6 and 7) in caller-owned device memory
   `d_storage` (>= storage bytes, 256-byte aligned; must outlive the table)
   and initialise it to empty on `stream`.  Geometry: 1 <= bins < 2^32 and bins >= d; slots_per_bin in
   {1, 2, 4, 8}; d in {2, 3, 4}; d > 2 needs slots_per_bin == 1; CK_RATTLE needs
   slots_per_bin == 1; CK_QUEUE and ghosts need d == 2.  The library allocates
   its own round scratch with hipMalloc (released by ck_destroy). */
ck_status ck_create(uint64_t bins, uint32_t slots_per_bin, uint32_t d, ck_scheme scheme,
                    const ck_options* opt, void* d_storage, size_t storage_bytes,
                    void* stream, ck_table** out);

/* Empty the table (every slot, metadata and claim word), zero its counters and
   restart its insert-op count, on `stream`; storage and scratch are kept.
   After it the table is the empty table of Sec. 3's experiments (every
   experiment fills from empty).  Errors: CK_EINVAL for a null handle. */
ck_status ck_clear(ck_table* t, void* stream);

/* Insert n keys with their values (8-byte values, 4-byte for single-slot
   bins).  Keys must be absent from the table and distinct within the call
   (Sec. 3: inserts do not check for presence); violating this is undefined.
   d_status[i] receives a CK_OP_* byte.  Sub-batches of batch_ops ops run the
   round protocol in order. */
ck_status ck_insert(ck_table* t, const uint64_t* d_keys, const void* d_vals, uint64_t n,
                    uint8_t* d_status, void* stream);

/* ck_insert plus per-op diagnostics (each may be NULL): bins viewed by the
   deciding plan, kicks of the committed chain, rounds lost to claims. */
ck_status ck_insert_ex(ck_table* t, const uint64_t* d_keys, const void* d_vals, uint64_t n,
                       uint8_t* d_status, uint32_t* d_views, uint32_t* d_kicks,
                       uint32_t* d_retries, void* stream);

/* Lookup (Sec. 1): probe the key's bins in hash order.  d_vals_out gets the
   value (0 when absent), d_found 1/0.  Fully asynchronous on `stream`. */
ck_status ck_lookup(ck_table* t, const uint64_t* d_keys, uint64_t n, void* d_vals_out,
                    uint8_t* d_found, void* stream);

/* Lookup with an explicit lanes-per-probe (1 or slots_per_bin); 0 = auto. */
ck_status ck_lookup_lpp(ck_table* t, const uint64_t* d_keys, uint64_t n, void* d_vals_out,
                        uint8_t* d_found, uint32_t lanes_per_probe, void* stream);

/* Delete (Sec. 1): empty every slot holding the key (both copies of a ghost
   pair).  d_found gets CK_OP_OK / CK_OP_NOT_FOUND / CK_OP_ABORTED /
   CK_OP_BAD_KEY.  Deleting one key twice in a call: the first op finds it. */
ck_status ck_delete(ck_table* t, const uint64_t* d_keys, uint64_t n, uint8_t* d_found,
                    void* stream);

/* For callers that cannot allocate device memory (serving loops and harnesses
   that forbid hipMalloc after set-up): ck_delete, with every round scratch
   array (pending lists, plan headers, inline moves, per-op counters, round
   counters, statistics staging) carved from one fixed array of
   CK_NOALLOC_SCRATCH_BYTES that the library holds per device (until the
   process ends) instead of the table's own scratch.  It calls no hipMalloc,
   hipFree or allocating routine; its results (d_found, the table, every
   counter) equal ck_delete's for the same table and keys.  A sub-batch
   (min(n, batch_ops) ops) may hold at most CK_NOALLOC_MAX_OPS ops, else
   CK_EINVAL before any device work.  Every call on one device shares that
   device's array: calls that overlap on one device (other streams, other host
   threads) race and must not be made; consecutive calls are safe, since each
   returns with its work complete.  Kernel-class timing is not recorded. */
#define CK_NOALLOC_MAX_OPS 65536u
#define CK_NOALLOC_SCRATCH_BYTES (5u << 20)
ck_status ck_delete_noalloc(ck_table* t, const uint64_t* d_keys, uint64_t n, uint8_t* d_found,
                            void* stream);

/* Overwrite (Sec. 1: constant-time overwrites): a stored key gets the new
   value (8 bytes, or 4 for single-slot bins) in every slot holding it; its
   key, ghost mark and rattle counter stay.  An absent key is not inserted.
   d_found gets CK_OP_OK / CK_OP_NOT_FOUND / CK_OP_ABORTED / CK_OP_BAD_KEY.  A
   key given twice in a call keeps the later op's value.  No counter of
   ck_stats changes. */
ck_status ck_overwrite(ck_table* t, const uint64_t* d_keys, const void* d_vals, uint64_t n,
                       uint8_t* d_found, void* stream);

/* Upsert (Sec. 1, inserts next to constant-time overwrites): each op first
   looks for its key in the key's bins, in hash order.  A stored key gets the
   new value in place, as ck_overwrite, and d_status[i] = CK_OP_UPDATED; an
   absent key is inserted with the table's scheme (CK_OP_OK / FAIL_CHAIN /
   ABORTED), and its plan also claims the key's first bin, so that a key given
   several times in one call is inserted by its first op and overwritten by the
   later ones, in op order.  Keys need not be absent or distinct.  The
   diagnostics (each may be NULL) are ck_insert_ex's; an absent key's views
   include the H bins of the presence check, a found key's are the bins
   searched up to it.  Updated ops count in no ck_stats counter; the others
   count as inserts, and the call adds n to the insert-op count. */
ck_status ck_upsert(ck_table* t, const uint64_t* d_keys, const void* d_vals, uint64_t n,
                    uint8_t* d_status, uint32_t* d_views, uint32_t* d_kicks,
                    uint32_t* d_retries, void* stream);

/* Transactional batch (Sec. 8): n_txn transactions, transaction t being the
   operations [d_txn_off[t], d_txn_off[t + 1]) of d_kind / d_keys / d_vals
   (d_txn_off holds n_txn + 1 increasing indices; kinds CK_TXN_*; values are
   read for inserts and overwrites).  Each transaction is applied atomically:
   its operations run in order, each seeing the earlier ones' writes (an
   insert runs the table's kick-out walk, chain included), and the table ends
   as if the committed transactions had run one at a time (Sec. 8's
   transactional correctness).  Transactions run in sub-batches in rounds:
   every pending transaction plans against the round's snapshot and claims
   every bin it reads or writes (its read and write sets, the claim flags of
   Sec. 8.2; the smallest transaction index wins a bin); one that owns all its
   bins commits, the others plan again next round.  A transaction whose plan
   would touch more than CK_TXN_MAX_BINS bins, or that loses max_rounds rounds
   (when set), aborts.  Per op, d_status: lookups, deletes and overwrites
   CK_OP_OK (found) or CK_OP_NOT_FOUND; inserts CK_OP_OK or CK_OP_FAIL_CHAIN;
   every op of an aborted transaction CK_OP_ABORTED; CK_OP_BAD_KEY for the
   reserved key.  d_vals_out[j]: a lookup's value (0 otherwise).
   d_txn_round[t]: the round (within its sub-batch, from 0) in which t
   committed or aborted.  Inserted keys must be absent and inserted once.
   Tables: CK_RANDOM_WALK or CK_QUEUE, d == 2, slots_per_bin 2, 4 or 8, no
   ghosts, no stash, uniform hashes; else CK_EUNSUPPORTED.  The library
   allocates the transactions' scratch (per lane of a sub-batch of at most
   2^14 transactions: CK_TXN_MAX_BINS bins and an undo log of max_chain + 2
   records) on the first call.  Synchronises `stream` once per round. */
enum { CK_TXN_LOOKUP = 0, CK_TXN_INSERT = 1, CK_TXN_DELETE = 2, CK_TXN_OVERWRITE = 3 };
#define CK_TXN_MAX_BINS 512u
ck_status ck_transact(ck_table* t, const uint8_t* d_kind, const uint64_t* d_keys,
                      const uint64_t* d_vals, const uint32_t* d_txn_off, uint32_t n_txn,
                      uint8_t* d_status, uint64_t* d_vals_out, uint32_t* d_txn_round,
                      void* stream);

/* Copy the counters to host memory (synchronises `stream`).  The counters are
   the paper's cost measures: bins viewed per insertion by density (Sec. 3),
   kick-out chain lengths (Sec. 5), failures, and the rounds lost to claims
   (Sec. 8.2).  Errors: CK_EINVAL for a null handle or `h_out`; CK_EDEVICE when
   the copy fails.  ck_stats_reset zeroes them (not `stored`). */
ck_status ck_stats_get(ck_table* t, ck_stats* h_out, void* stream);
ck_status ck_stats_reset(ck_table* t, void* stream);

/* Per-kernel timing, measured with HIP events on the caller's stream around
   every launch of each enabled kernel class (enabling resets it).  Two events
   per timed launch: time only the classes of interest in timed runs. */
typedef struct {
  uint64_t launches;
  double ms;            /* summed launch durations */
} ck_kernel_time;

typedef struct {
  ck_kernel_time plan_fresh;  /* placement without eviction, every pending op */
  ck_kernel_time plan_evict;  /* kick-out planners: walk (random/queue/rattle) or search */
  ck_kernel_time plan_delete;
  ck_kernel_time commit;      /* claim check, reverse-order writes, metadata, next list */
  ck_kernel_time stats;       /* density bands and totals */
  ck_kernel_time lookup;
  uint64_t evict_views;       /* bins viewed by the kick-out planners while enabled */
} ck_timing;

/* Classes to time (bit mask for ck_timing_enable); 0 turns timing off. */
enum {
  CK_TIME_PLAN_FRESH = 1, CK_TIME_PLAN_EVICT = 2, CK_TIME_PLAN_DELETE = 4, CK_TIME_COMMIT = 8,
  CK_TIME_STATS = 16, CK_TIME_LOOKUP = 32, CK_TIME_ALL = 63
};
ck_status ck_timing_enable(ck_table* t, uint32_t class_mask);
/* Synchronises `stream`, then copies the timing gathered since enabling. */
ck_status ck_timing_get(ck_table* t, ck_timing* h_out, void* stream);

/* Canonical image of the table in host memory, the same layout the oracle
   writes, so two images compare byte for byte: per slot key (Sec. 1), value
   (zero extended for 32-bit values) and rattle counter (Sec. 7); per bin the
   metadata word (duplicate marks, Sec. 4; spawn count, Sec. 5; hit counter,
   Sec. 6)
     bits 0-7 duplicate marks, bits 8-11 spawn count, bits 24-31 hit counter.
   Arrays hold bins*slots_per_bin (keys, vals, rattle) and bins (meta)
   entries.  Export synchronises `stream`; import recomputes `stored`. */
ck_status ck_export(ck_table* t, uint64_t* h_keys, uint64_t* h_vals, uint16_t* h_rattle,
                    uint32_t* h_meta, void* stream);
ck_status ck_import(ck_table* t, const uint64_t* h_keys, const uint64_t* h_vals,
                    const uint16_t* h_rattle, const uint32_t* h_meta, void* stream);

/* The stash (Sec. 2) in host memory: `stash` keys and values, entry by entry
   (key CK_EMPTY_KEY: free; values zero extended).  Export synchronises
   `stream`; import (after ck_import) adds the stashed keys to `stored`.
   CK_EINVAL when the table has no stash. */
ck_status ck_export_stash(ck_table* t, uint64_t* h_keys, uint64_t* h_vals, void* stream);
ck_status ck_import_stash(ck_table* t, const uint64_t* h_keys, const uint64_t* h_vals,
                          void* stream);

/* Hash a key as the table does: its d distinct bin indices h_0..h_{d-1}, in
   order (Sec. 1, Sec. 7).  Host arithmetic, no device call. */
ck_status ck_hash(const ck_table* t, uint64_t key, uint64_t* h_bins_out);

/* Number of insert ops submitted so far (the id of the next insert op). */
uint64_t ck_insert_count(const ck_table* t);

/* Release the handle and the library's scratch; the caller's storage is not
   freed.  Synchronises the device.  Not a paper operation: resource
   management of the C ABI.  Errors: CK_EINVAL for a null handle. */
ck_status ck_destroy(ck_table* t);

/* ---- groups: many independent tables of uneven sizes served together ----
   Not a paper operation: the batched form of the calls above (the paper's
   tables, Sec. 1, many at once), for callers that hold many small tables.
   A group holds n_tables tables (bins[i] bins each; same slots_per_bin, d,
   scheme and options) in one caller allocation.  Every op names its table
   (d_table[i] < n_tables); one call serves ops of any mix of tables with the
   same launches, and its results equal those of per-table calls: a table's
   ops in one sub-batch of the call (batch_ops ops of the whole call) form that
   table's sub-batch, in call order.  The random walk's choices are keyed by
   the op's index in the group's stream of inserts.  Tables never interact:
   each table's bins are a disjoint range of the group's bin array.  Counters
   are kept for the group as a whole (no density bands). */
typedef struct ck_group ck_group;

ck_status ck_group_storage_bytes(uint32_t n_tables, const uint64_t* h_bins,
                                 uint32_t slots_per_bin, uint32_t d, size_t* out);
ck_status ck_group_create(uint32_t n_tables, const uint64_t* h_bins, uint32_t slots_per_bin,
                          uint32_t d, ck_scheme scheme, const ck_options* opt, void* d_storage,
                          size_t storage_bytes, void* stream, ck_group** out);
/* Insert; d_views, d_kicks, d_retries may be NULL. */
ck_status ck_group_insert(ck_group* g, const uint32_t* d_table, const uint64_t* d_keys,
                          const void* d_vals, uint64_t n, uint8_t* d_status, uint32_t* d_views,
                          uint32_t* d_kicks, uint32_t* d_retries, void* stream);
ck_status ck_group_lookup(ck_group* g, const uint32_t* d_table, const uint64_t* d_keys,
                          uint64_t n, void* d_vals_out, uint8_t* d_found,
                          uint32_t lanes_per_probe, void* stream);
ck_status ck_group_delete(ck_group* g, const uint32_t* d_table, const uint64_t* d_keys,
                          uint64_t n, uint8_t* d_found, void* stream);
ck_status ck_group_overwrite(ck_group* g, const uint32_t* d_table, const uint64_t* d_keys,
                             const void* d_vals, uint64_t n, uint8_t* d_found, void* stream);
/* Upsert (as ck_upsert); d_views, d_kicks, d_retries may be NULL. */
ck_status ck_group_upsert(ck_group* g, const uint32_t* d_table, const uint64_t* d_keys,
                          const void* d_vals, uint64_t n, uint8_t* d_status, uint32_t* d_views,
                          uint32_t* d_kicks, uint32_t* d_retries, void* stream);
/* One table's stash (as ck_export_stash). */
ck_status ck_group_export_stash(ck_group* g, uint32_t table, uint64_t* h_keys, uint64_t* h_vals,
                                void* stream);
/* Canonical image of one table of the group (as ck_export). */
ck_status ck_group_export_table(ck_group* g, uint32_t table, uint64_t* h_keys, uint64_t* h_vals,
                                uint16_t* h_rattle, uint32_t* h_meta, void* stream);
ck_status ck_group_stats_get(ck_group* g, ck_stats* h_out, void* stream);
ck_status ck_group_timing_enable(ck_group* g, uint32_t class_mask);
ck_status ck_group_timing_get(ck_group* g, ck_timing* h_out, void* stream);
ck_status ck_group_clear(ck_group* g, void* stream);
uint64_t ck_group_insert_count(const ck_group* g);
ck_status ck_group_destroy(ck_group* g);

const char* ck_strerror(ck_status s);

#ifdef __cplusplus
}
#endif
#endif /* CK_H */
