// ck_internal.h -- device-side data layout and kernel launchers of libck.
//
// HBM layout of one table (caller storage, each array 256-byte aligned):
//   slots  bins*B x 16 B   {u64 key, u64 aux}; B >= 2: aux = value;
//                          B == 1: aux = value(32) | rattle(16) << 32
//   meta   bins x 4 B      bits 0-7 duplicate marks, 8-11 spawn count,
//                          24-31 hit counter
//   owner  bins x 8 B      claim word of the round protocol:
//                          (~epoch) << 32 | op index; the smallest word wins,
//                          so a newer round always overrides an older one.
// A bin of B >= 4 slots is one 64- or 128-byte line: one probe is one
// coalesced HBM transaction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ck.h"

namespace ck {

constexpr uint64_t kEmpty = CK_EMPTY_KEY;
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Move flags: one entry of a plan (a write to one slot, or a mark update).
enum : uint8_t {
  MV_SUPERSEDED = 1,  // a later move of the same plan rewrites this slot
  MV_DUP = 2,         // the written record is a ghost duplicate
  MV_HC = 4,          // the write is an insertion counted by the hit counter
  MV_DUPCLR = 8,      // no slot write: clear the duplicate mark only (ghost twin)
  MV_CLEAR = 16,      // delete: the slot becomes empty
  MV_VALUE = 32,      // overwrite: only the value changes (key, mark and, in a
                      // single-slot bin, the rattle counter stay)
};

struct Move {            // 24 bytes
  uint64_t key;
  uint64_t aux;
  uint32_t bin;
  uint8_t slot;
  uint8_t flags;
  uint16_t pad;
};

// A move stored inline with its op: the written record is the op's own key
// and value (or nothing, for clears and duplicate-mark updates).
struct IMove {           // 8 bytes
  uint32_t bin;
  uint32_t sf;           // slot | flags << 8
};

enum : uint32_t {
  PL_FAIL = 0, PL_OK = 1, PL_EVICT = 2, PL_NOTFOUND = 3, PL_UPDATED = 4, PL_STASHED = 5
};

// Plan of one op of the sub-batch: a 16-byte header (one load in the commit
// kernel), in an array of its own so that the headers of consecutive ops fill
// whole lines.  Plans of at most three moves that write only the op's own
// record keep them inline: the first in the header, the others in the per-op
// inline array.  The header is
//   inline plans (fresh placements, deletes, overwrites):
//     {st, views, first move's bin, first move's slot | flags << 8};
//   arena plans (kick-out chains, kHdrArena set in st):
//     {st, views, arena offset of the moves, kicks};
// with st = status | twins << 4 | n_moves << 8 | flags (bits 28-30).  Arena
// plans also have a spawn record {n_spawn, spawn_off} (sorted search: the
// plan's spawn list in the spawn arena) in a second per-op array.
constexpr uint32_t kHdrArena = 1u << 28;
// Upsert of an absent key: the plan also holds a claim on the key's first bin
// (which it may not write), so that two upserts of one new key conflict.
constexpr uint32_t kHdrKeyClaim = 1u << 29;
// The plan writes one stash entry, whose index (in the stash array of every
// table) is the header's fourth word; it claims that entry like a bin.
constexpr uint32_t kHdrStash = 1u << 30;
constexpr uint32_t kMaxStash = 64;  // stash entries per table
constexpr uint32_t kExtraInline = 2;  // inline moves beyond the first, per op

// Lanes per op in the fresh planner: each lane holds B / lanes consecutive
// slots of a bin, so a wavefront keeps more ops (and their dependent bin
// reads) in flight than with one lane per slot.
__host__ __device__ constexpr int fresh_lanes(int B) { return B >= 4 ? B / 2 : B; }
__host__ __device__ inline uint32_t hdr_pack(uint32_t status, uint32_t twins, uint32_t nm) {
  return status | (twins << 4) | (nm << 8);
}

// Pending lists.  After the first round of a sub-batch (whose list is every
// op in order), the ops that go again are listed by the commit kernel in
// kStripes segments: commit wavefront u (kCommitWaveOps consecutive
// positions) appends its ops to segment u % kStripes with one atomic add on
// that segment's count, so the adds spread over kStripes counters (each on
// its own 128-byte line).  A list of n ops has positions 0..n-1 through the
// prefix sums of the counts.  The order within a list is immaterial: every
// kernel's result for an op depends on the op, never on its position.
constexpr uint32_t kStripes = 64;
constexpr uint32_t kStripeWords = 32;
constexpr uint32_t kCommitLanes = 2;                    // lanes per plan in the commit kernel
constexpr uint32_t kCommitOps = 256 / kCommitLanes;     // plans per commit workgroup pass
constexpr uint32_t kCommitWaveOps = 64 / kCommitLanes;  // plans per commit wavefront
__host__ __device__ inline uint32_t stripe_capacity(uint32_t m) {
  const uint32_t waves = (m + kCommitWaveOps - 1) / kCommitWaveOps;
  return (waves + kStripes - 1) / kStripes * kCommitWaveOps;
}

struct Ctr {             // device counters of the round loop
  uint32_t overflow;     // a planner ran out of arena this round (round is void)
  uint32_t overflow_seen;  // sticky: some earlier round of the sub-batch was void
  uint32_t rounds;       // rounds that committed (not void, ops pending)
  uint32_t unfinished;   // set by the statistics: the sub-batch (or the one
                         // before it) still had pending ops, nothing applied
  uint32_t pad[28];
  uint32_t cnt[2][kStripes * kStripeWords];  // segment counts of pending list p
};

// What the host needs of a sub-batch after its enqueued rounds, written by the
// first statistics kernel straight into pinned host memory (no copy launch):
// whether its last list came out empty, the arena-overflow flags and the
// rounds that committed.
struct HostSum {
  uint32_t done, overflow, overflow_seen, rounds;
};

// Device accumulators (they mirror ck_stats), in kStatStripes copies:
// workgroup w adds into copy w % kStatStripes, so the few adds per workgroup
// of a statistics or lookup launch spread over separate lines instead of
// serialising on one; readers sum the copies (`stored` included).
constexpr int kStatStripes = 16;
enum {
  S_INS_OK, S_INS_FAIL, S_INS_ABORT, S_INS_BAD, S_VIEWS, S_VIEWS_ALL, S_KICKS, S_MAX_KICKS,
  S_RETRIES, S_ROUNDS, S_TWINS, S_LOOKUPS, S_LOOKUP_HITS, S_LOOKUP_PROBES, S_DELETES,
  S_DEL_FOUND, S_DEL_PROBES, S_DEL_RETRIES, S_STORED, S_INS_STASHED,
  S_NUM  // the number of scalar counters
};
struct DevStatLine {
  unsigned long long v[S_NUM];
  unsigned long long pad[32 - S_NUM];  // 256 bytes
  unsigned long long band[4][CK_BANDS];
};
struct DevStats {
  DevStatLine s[kStatStripes];
};

// A table's bin range inside the bin array (a group of tables shares one).
struct Tab {
  uint32_t base, n;
};

// Everything a kernel needs about a table, passed by value.
struct Geo {
  uint64_t a[4], c[4];
  ulonglong2* slots;
  uint32_t* meta;
  unsigned long long* owner;
  uint32_t n;            // bins (< 2^32)
  uint32_t B, H, scheme;
  uint32_t ghost, balance, max_chain, max_search;
  uint64_t rng_seed;
  // the stash (Sec. 2): stash_n entries per table, table t's at t * stash_n;
  // a claim word per entry and a count of used entries per table
  ulonglong2* stash;
  unsigned long long* stash_owner;
  uint32_t* stash_cnt;
  uint32_t stash_n;
  uint32_t stash_tables;
  uint32_t hash_bias;  // 0: uniform hashes; 1-4: biased
  uint32_t spawn_k;    // > 1: BFS / sorted search spawn this many records at a time
};

// Round-scratch pointers of one sub-batch.
struct Round {
  const uint64_t* keys;      // sub-batch keys
  const void* vals;          // sub-batch values (8 or 4 bytes each)
  const uint32_t* op_table;  // group mode: table index of each op (else null)
  const uint2* tdesc;        // group mode: {bin base, bins} of each table
  const uint32_t* pend;      // this round's pending list (segments of stripe_cap)
  const uint32_t* pcnt;      // its segment counts; null in the first round
  uint32_t npend;            // first round: the op count; later rounds: the size
                             // the grids are made for (kernels loop past it)
  uint32_t stripe_cap;       // entries per list segment
  uint32_t* next;            // the next round's list: ops that go again
  uint32_t* next_cnt;        // its segment counts (zeroed by this round's planner)
  const uint32_t* gate;      // the previous sub-batch's `unfinished` flag, or
                             // null: while it is set, every kernel of this round
                             // does nothing (the host enqueues one sub-batch ahead)
  uint32_t* evict;           // ops that need an eviction plan: fresh-planner
                             // wavefront u (positions [u opw, (u + 1) opw),
                             // opw = 64 / fresh_lanes(B)) puts its
                             // evict_cnt[u] ops at evict[u opw ...)
  uint32_t* evict_cnt;       // per fresh-planner wavefront
  uint4* hdr;                // per op: the plan header
  uint2* hdr_spawn;          // per op: arena plans' spawn record
  IMove* imv;                // kExtraInline per op
  Move* arena;
  uint32_t arena_cap;
  uint32_t* spawns;
  uint32_t spawn_cap;
  Ctr* ctr;
  uint64_t op_base;          // global insert index of op 0 of the sub-batch
  unsigned long long tag;    // (~epoch) << 32
  uint8_t* status;           // caller's per-op status (sub-batch view)
  uint32_t* op_views;         // bins viewed by the deciding plan
  uint32_t* op_lost;          // bins viewed by plans that lost their claims
  uint32_t* op_kicks;
  uint32_t* op_retries;
  uint32_t* op_twins;
  uint32_t max_rounds;
  uint32_t is_delete;         // the delete planner: deletes, and overwrites when
  uint32_t overwrite;         // this is set (new values in place)
  uint32_t upsert;            // inserts that first look for the key (found: new value)
  uint32_t first;            // first round of the sub-batch: pend[p] = p, counters unset
  unsigned long long* wg_views;  // per eviction workgroup: bins viewed (cumulative)
  void* wg_scratch;          // per-workgroup scratch of the eviction planners
  uint32_t wg_scratch_bytes;
  DevStats* stats;
  HostSum* hsum;             // pinned host memory of the sub-batch's counter set
};

// One round of a transactional batch (Sec. 8): the pending transactions of a
// sub-batch, one lane each.
constexpr uint32_t kTxnBins = CK_TXN_MAX_BINS;  // bins one transaction's plan may touch
enum : uint32_t { TXN_LOOKUP = CK_TXN_LOOKUP, TXN_INSERT = CK_TXN_INSERT,
                  TXN_DELETE = CK_TXN_DELETE, TXN_OVERWRITE = CK_TXN_OVERWRITE };
struct TxnRound {
  const uint8_t* kind;       // per op
  const uint64_t* keys;
  const uint64_t* vals;
  const uint32_t* off;       // transaction t: ops [off[t], off[t + 1])
  uint32_t t0;               // first transaction of the sub-batch
  const uint32_t* pend;      // pending transactions (within the sub-batch); null: 0..npend-1
  uint32_t npend;
  uint32_t* next;            // the transactions that go again, and their count
  uint32_t* next_cnt;
  uint8_t* status;           // per op
  uint64_t* vout;            // per op: a lookup's value
  uint32_t* txn_round;       // per transaction: the round it committed or aborted in
  uint32_t* lost;            // per transaction of the sub-batch: rounds lost
  uint32_t* nob;             // per pending position: overlay entries, kNone: too many bins
  uint32_t round, max_rounds;
  uint64_t op_base;          // the insert-op index of op 0 (random walk draws)
  unsigned long long tag;    // (~epoch) << 32
  char* scratch;             // per pending position: lane_bytes of overlay and undo log
  uint32_t lane_bytes, undo_cap;
  DevStats* stats;
};

// ---- launchers (ck_kernels.hip) ----
hipError_t launch_init(const Geo& g, hipStream_t s);
hipError_t launch_lookup(const Geo& g, const uint64_t* keys, uint64_t n, void* vals_out,
                         uint8_t* found, uint32_t lpp, DevStats* st, const uint32_t* op_table,
                         const uint2* tdesc, hipStream_t s);
hipError_t launch_plan_fresh(const Geo& g, const Round& r, hipStream_t s);
hipError_t launch_plan_evict(const Geo& g, const Round& r, uint32_t grid, hipStream_t s);
hipError_t launch_plan_delete(const Geo& g, const Round& r, hipStream_t s);
hipError_t launch_commit(const Geo& g, const Round& r, hipStream_t s);
// Sub-batch statistics; they apply only if the pending list whose segment
// counts `open` points to is empty and the flag `r.gate` points to is clear
// (else the kernels return at once and the host enqueues them again later).
// The first statistics kernel records the outcome in r.ctr->unfinished.
hipError_t launch_batch_stats(const Round& r, uint64_t m, uint64_t slots, uint32_t* block_tmp,
                              uint32_t is_delete, const uint32_t* open, hipStream_t s);
// 32-bit words of `block_tmp` that the statistics of a sub-batch of m ops use.
size_t stats_tmp_words(uint64_t m);
size_t evict_lds_bytes(const Geo& g);
int evict_resident_per_cu(const Geo& g);
size_t evict_wg_scratch_bytes(const Geo& g);
hipError_t launch_export_meta(const Geo& g, hipStream_t s);
size_t txn_lane_bytes(const Geo& g);
uint32_t txn_undo_cap(const Geo& g);
hipError_t launch_txn(const Geo& g, const TxnRound& r, bool commit, hipStream_t s);
// p[0..count) = value (a small fill kernel; no memset node)
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s);

}  // namespace ck
