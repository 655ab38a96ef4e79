// ck_api.hip -- host runtime of libck: table objects, the round driver and the
// C ABI declared in include/ck.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ck_internal.h"

using namespace ck;

// Event timing of kernel classes (opt-in).  Pairs of events are recorded
// around launches and resolved after the stream has been synchronised.
enum TimedKind { TK_FRESH, TK_EVICT, TK_DELETE, TK_COMMIT, TK_STATS, TK_LOOKUP, TK_N };
struct Timer {
  bool on = false;
  uint32_t mask = 0;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[TK_N] = {0};
  uint64_t launches[TK_N] = {0};
  uint64_t views_base = 0, views_acc = 0;
  hipEvent_t take() {
    if (pool.empty()) {
      // timing only: no system-scope fence when the event is recorded, so an
      // event costs less and disturbs the launches around it less
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t begin(hipStream_t s, int kind) {
    if (!on || !(mask & (1u << kind))) return nullptr;
    hipEvent_t e = take();
    if (e) (void)hipEventRecord(e, s);
    return e;
  }
  void end(int kind, hipEvent_t b, hipStream_t s) {
    if (!on || !b) return;
    hipEvent_t e = take();
    if (!e) return;
    (void)hipEventRecord(e, s);
    pending.push_back({kind, {b, e}});
  }
  // Resolves the pairs whose end event has completed (pairs complete in the
  // order they were recorded); later pairs stay pending.
  void collect() {
    size_t k = 0;
    for (; k < pending.size(); ++k) {
      auto& p = pending[k];
      if (hipEventQuery(p.second.second) == hipErrorNotReady) break;
      float t = 0;
      if (hipEventElapsedTime(&t, p.second.first, p.second.second) == hipSuccess) {
        ms[p.first] += t;
        launches[p.first] += 1;
      }
      pool.push_back(p.second.first);
      pool.push_back(p.second.second);
    }
    pending.erase(pending.begin(), pending.begin() + k);
  }
  void reset() {
    collect();
    for (int k = 0; k < TK_N; ++k) { ms[k] = 0; launches[k] = 0; }
  }
  ~Timer() {
    for (auto& p : pending) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct ck_table {
  Geo g;
  ck_options opt;
  uint64_t bins;
  uint32_t B, H;
  ck_scheme scheme;
  uint64_t insert_count = 0;
  uint32_t epoch = 0;
  // round scratch
  uint32_t batch_cap = 0;
  uint32_t* pend[2] = {nullptr, nullptr};
  uint4* hdr = nullptr;
  uint2* hdr_spawn = nullptr;
  IMove* imv = nullptr;
  uint32_t* evict = nullptr;
  uint32_t* evict_cnt = nullptr;
  Move* arena = nullptr;
  uint32_t arena_cap = 0;
  uint32_t* spawns = nullptr;
  uint32_t spawn_cap = 0;
  uint32_t* op[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // views, lost, kicks, retries, twins
  unsigned long long* wg_views = nullptr;  // per eviction workgroup: bins viewed
  Ctr* ctr = nullptr;    // two sets: sub-batches alternate between them
  HostSum* h_sum = nullptr;  // pinned: what the host needs of each set's sub-batch
  hipEvent_t ctr_ready[2] = {nullptr, nullptr};  // a set's summary has landed
  void* wg_scratch = nullptr;
  uint32_t wg_bytes = 0;
  uint32_t evict_grid = 0;
  DevStats* dstats = nullptr;
  uint32_t* block_tmp = nullptr;
  uint32_t stripe_cap = 0;  // entries per pending-list segment
  // rounds the last two insert sub-batches took (the larger sizes the next
  // enqueue) and the rounds the last delete sub-batch took
  uint32_t tail_hint = 2;
  uint32_t tail_prev = 2;
  uint32_t tail_hint_del = 1;
  // upserts keep their own history: their key claims make them take more
  // rounds than the table's plain inserts
  uint32_t tail_hint_ups = 2;
  uint32_t tail_prev_ups = 2;
  // host-side counters
  uint64_t rounds = 0, lookups = 0;
  Timer timer;
  // transactional batches: per-lane scratch and lists, allocated on first use
  char* txn_scratch = nullptr;
  uint32_t txn_cap = 0;
  uint32_t* txn_list[2] = {nullptr, nullptr};
  uint32_t* txn_nob = nullptr;
  uint32_t* txn_lost = nullptr;
  uint32_t* txn_cnt = nullptr;
};

// The round scratch one call runs on: the table's own arrays (allocated at
// create; the plan arena grows when a round runs out), or a fixed set carved
// from the library's static array, which never grows.
struct Scratch {
  uint32_t* pend[2];
  uint4* hdr;
  uint2* hdr_spawn;
  IMove* imv;
  uint32_t* evict;
  uint32_t* evict_cnt;
  Move* arena;
  uint32_t arena_cap;
  uint32_t* spawns;
  uint32_t spawn_cap;
  uint32_t* op[5];
  Ctr* ctr;
  uint32_t* block_tmp;
  uint32_t stripe_cap;
  bool fixed;  // no growth: an overflowing round is an error
};

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Scratch own_scratch(const ck_table* t) {
  Scratch x{};
  x.pend[0] = t->pend[0];
  x.pend[1] = t->pend[1];
  x.hdr = t->hdr;
  x.hdr_spawn = t->hdr_spawn;
  x.imv = t->imv;
  x.evict = t->evict;
  x.evict_cnt = t->evict_cnt;
  x.arena = t->arena;
  x.arena_cap = t->arena_cap;
  x.spawns = t->spawns;
  x.spawn_cap = t->spawn_cap;
  for (int k = 0; k < 5; ++k) x.op[k] = t->op[k];
  x.ctr = t->ctr;
  x.block_tmp = t->block_tmp;
  x.stripe_cap = t->stripe_cap;
  x.fixed = false;
  return x;
}

// splitmix64 (Steele, Lea, Flood): derives the hash multipliers from the seed.
uint64_t sm_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Layout {
  size_t slots, meta, owner, total;
};
Layout layout(uint64_t bins, uint32_t B) {
  Layout L;
  L.slots = 0;
  L.meta = align256(bins * B * 16);
  L.owner = L.meta + align256(bins * 4);
  L.total = L.owner + align256(bins * 8);
  return L;
}

bool geometry_ok(uint64_t bins, uint32_t B, uint32_t d) {
  if (bins == 0 || bins >= (1ull << 32) || bins < d) return false;
  if (!(B == 1 || B == 2 || B == 4 || B == 8)) return false;
  if (d < 2 || d > 4) return false;
  if (d > 2 && B != 1) return false;
  return true;
}

#define HIP_TRY(x)                         \
  do {                                     \
    if ((x) != hipSuccess) return CK_EDEVICE; \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

void free_scratch(ck_table* t) {
  (void)hipFree(t->pend[0]);
  (void)hipFree(t->pend[1]);
  (void)hipFree(t->hdr);
  (void)hipFree(t->hdr_spawn);
  (void)hipFree(t->imv);
  (void)hipFree(t->evict);
  (void)hipFree(t->evict_cnt);
  (void)hipFree(t->arena);
  (void)hipFree(t->spawns);
  for (auto& p : t->op) (void)hipFree(p);
  (void)hipFree(t->ctr);
  if (t->h_sum) (void)hipHostFree(t->h_sum);
  for (auto& e : t->ctr_ready)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(t->wg_scratch);
  (void)hipFree(t->wg_views);
  (void)hipFree(t->dstats);
  (void)hipFree(t->block_tmp);
  (void)hipFree(t->g.stash);
  (void)hipFree(t->g.stash_owner);
  (void)hipFree(t->g.stash_cnt);
  (void)hipFree(t->txn_scratch);
  (void)hipFree(t->txn_list[0]);
  (void)hipFree(t->txn_list[1]);
  (void)hipFree(t->txn_nob);
  (void)hipFree(t->txn_lost);
  (void)hipFree(t->txn_cnt);
}

ck_status alloc_scratch(ck_table* t) {
  const uint32_t m = t->opt.batch_ops;
  t->batch_cap = m;
  // persistent eviction planners: as many one-wavefront workgroups as can be
  // resident at once (registers, LDS, wave slots), so no workgroup waits for
  // another to finish; when the query fails, as many as the LDS of a CU holds
  // (160 KiB on gfx950), at most 32
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t lds = evict_lds_bytes(t->g);
  size_t per_cu = std::max<size_t>(1, std::min<size_t>(32, (160 * 1024) / std::max<size_t>(lds, 1)));
  const int resident = evict_resident_per_cu(t->g);
  if (resident > 0) per_cu = std::min<size_t>(per_cu, (size_t)resident);
  if (t->opt.evict_wgs_per_cu) per_cu = std::min<size_t>(per_cu, t->opt.evict_wgs_per_cu);
  t->evict_grid = (uint32_t)(cus * per_cu);
  t->wg_bytes = (uint32_t)evict_wg_scratch_bytes(t->g);
  HIP_TRY(hipMalloc(&t->wg_scratch, (size_t)t->evict_grid * t->wg_bytes));
  HIP_TRY(dalloc(&t->wg_views, t->evict_grid));
  HIP_TRY(hipMemset(t->wg_views, 0, (size_t)t->evict_grid * 8));
  t->stripe_cap = stripe_capacity(m);
  HIP_TRY(dalloc(&t->pend[0], (size_t)kStripes * t->stripe_cap));
  HIP_TRY(dalloc(&t->pend[1], (size_t)kStripes * t->stripe_cap));
  HIP_TRY(dalloc(&t->hdr, m));
  HIP_TRY(dalloc(&t->hdr_spawn, m));
  HIP_TRY(dalloc(&t->imv, (size_t)m * kExtraInline));
  // evict regions: one per fresh-planner wavefront (64 / lanes-per-op ops),
  // every wavefront of the last pass included
  const size_t fl = fresh_lanes((int)t->B);
  const size_t evict_units = ((size_t)m * fl + 255) / 256 * 4;
  HIP_TRY(dalloc(&t->evict, evict_units * (64 / fl)));
  HIP_TRY(dalloc(&t->evict_cnt, evict_units));
  for (auto& p : t->op) HIP_TRY(dalloc(&p, m));
  // eviction plans sub-allocate from per-workgroup windows of 256 entries
  const uint64_t slack = (uint64_t)t->evict_grid * 512;
  t->arena_cap = (uint32_t)std::min<uint64_t>((uint64_t)m * 4 + slack, 1u << 30);
  HIP_TRY(dalloc(&t->arena, t->arena_cap));
  t->spawn_cap = (t->scheme == CK_SORTED || t->scheme == CK_HYBRID)
                     ? (uint32_t)std::min<uint64_t>((uint64_t)m * 2 + slack, 1u << 30)
                     : 16;
  HIP_TRY(dalloc(&t->spawns, t->spawn_cap));
  HIP_TRY(dalloc(&t->ctr, 2));
  HIP_TRY(hipMemset(t->ctr, 0, 2 * sizeof(Ctr)));
  HIP_TRY(hipHostMalloc((void**)&t->h_sum, 2 * sizeof(HostSum), hipHostMallocDefault));
  for (auto& e : t->ctr_ready) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIP_TRY(dalloc(&t->dstats, 1));
  HIP_TRY(hipMemset(t->dstats, 0, sizeof(DevStats)));
  HIP_TRY(dalloc(&t->block_tmp, stats_tmp_words(m)));
  // the stash: entries, their claim words, and a count per table
  if (t->g.stash_n) {
    const size_t ns = (size_t)t->g.stash_tables * t->g.stash_n;
    HIP_TRY(dalloc(&t->g.stash, ns));
    HIP_TRY(dalloc(&t->g.stash_owner, ns));
    HIP_TRY(dalloc(&t->g.stash_cnt, t->g.stash_tables));
  }
  return CK_OK;
}

ck_status grow_arena(ck_table* t) {
  HIP_TRY(hipDeviceSynchronize());
  (void)hipFree(t->arena);
  t->arena = nullptr;
  uint64_t nc = std::min<uint64_t>((uint64_t)t->arena_cap * 2, 1u << 30);
  t->arena_cap = (uint32_t)nc;
  HIP_TRY(dalloc(&t->arena, t->arena_cap));
  if (t->scheme == CK_SORTED || t->scheme == CK_HYBRID) {
    (void)hipFree(t->spawns);
    t->spawns = nullptr;
    t->spawn_cap = (uint32_t)std::min<uint64_t>((uint64_t)t->spawn_cap * 2, 1u << 30);
    HIP_TRY(dalloc(&t->spawns, t->spawn_cap));
  }
  return CK_OK;
}

Round make_round(ck_table* t, const Scratch& x, const uint64_t* keys, const void* vals,
                 uint8_t* status, uint32_t** ops, uint64_t op_base, bool is_delete,
                 const uint32_t* op_table, const uint2* tdesc) {
  Round r{};
  r.op_table = op_table;
  r.tdesc = tdesc;
  r.keys = keys;
  r.vals = vals;
  r.hdr = x.hdr;
  r.hdr_spawn = x.hdr_spawn;
  r.imv = x.imv;
  r.evict = x.evict;
  r.evict_cnt = x.evict_cnt;
  r.arena = x.arena;
  r.arena_cap = x.arena_cap;
  r.spawns = x.spawns;
  r.spawn_cap = x.spawn_cap;
  r.ctr = x.ctr;
  r.op_base = op_base;
  r.status = status;
  r.op_views = ops[0];
  r.op_lost = ops[1];
  r.op_kicks = ops[2];
  r.op_retries = ops[3];
  r.op_twins = ops[4];
  r.max_rounds = t->opt.max_rounds;
  r.is_delete = is_delete ? 1 : 0;
  r.wg_scratch = t->wg_scratch;
  r.wg_views = t->wg_views;
  r.wg_scratch_bytes = t->wg_bytes;
  r.stats = t->dstats;
  return r;
}

// The phased rounds of a sub-batch, then its statistics.  The first round's
// list is every op; each later round's list (and count) exists only on the
// device, so those rounds run capped grids that loop over whatever count
// they find.  For a sub-batch the host enqueues as many rounds as the larger
// of the last two insert sub-batches took (deletes: one more than the last
// delete sub-batch) and the statistics, whose first kernel writes the
// host's summary of the sub-batch into pinned memory, and does so one
// sub-batch ahead: sub-batch b + 1 is
// enqueued before the host waits for b's counters.  Every kernel of b + 1
// checks that b's last list came out empty (its gate) and otherwise does
// nothing; the host then runs more rounds of b and enqueues b + 1 again.
// The statistics of a sub-batch apply only when its own last list is empty
// too; their first kernel records the outcome in the `unfinished` flag that
// the next sub-batch's kernels read.  Sub-batches alternate between two sets
// of round counters.
constexpr uint32_t kMaxTailHint = 12;

// One sub-batch in flight, as the host tracks it.
struct Flight {
  Round r;
  uint64_t m = 0, slots = 0;
  int set = 0;          // its round-counter set
  int cur = 0;          // list parity its next round reads
  uint64_t guard = 0;   // rounds left before the loop counts as stuck
  bool live = false;
  const Scratch* fixed = nullptr;  // the call's fixed scratch, or null: the table's own
};

// The scratch a sub-batch runs on, read afresh (the table's arena may have grown).
Scratch scratch_of(const ck_table* t, const Flight& f) {
  return f.fixed ? *f.fixed : own_scratch(t);
}

ck_status enqueue_rounds(ck_table* t, Flight& f, uint32_t K, bool first, const uint32_t* gate,
                         hipStream_t s) {
  Timer& T = t->timer;
  Round& r = f.r;
  const Scratch x = scratch_of(t, f);
  Ctr* c = x.ctr + f.set;
  if (first) f.cur = 0;
  for (uint32_t k = 0; k < K; ++k) {
    // The lowest pending op always commits, so m rounds suffice; arena growth
    // adds a few void rounds.  Anything beyond that is a fault, not progress.
    if (f.guard == 0) return CK_EDEVICE;
    --f.guard;
    ++t->epoch;
    if (t->epoch == 0) {  // claim tags wrapped: reset every claim word
      HIP_TRY(hipMemsetAsync(t->g.owner, 0xFF, (size_t)t->bins * 8, s));
      if (t->g.stash_n)
        HIP_TRY(hipMemsetAsync(t->g.stash_owner, 0xFF,
                               (size_t)t->g.stash_tables * t->g.stash_n * 8, s));
      t->epoch = 1;
    }
    r.tag = (unsigned long long)(~t->epoch) << 32;
    r.first = first ? 1u : 0u;
    r.npend = (uint32_t)f.m;  // grid size; later rounds cap it
    r.ctr = c;
    r.hsum = t->h_sum + f.set;
    r.gate = gate;
    r.pend = x.pend[f.cur];
    r.pcnt = first ? nullptr : c->cnt[f.cur];
    r.next = x.pend[f.cur ^ 1];
    r.next_cnt = c->cnt[f.cur ^ 1];
    r.stripe_cap = x.stripe_cap;
    r.arena = x.arena;
    r.arena_cap = x.arena_cap;
    r.spawns = x.spawns;
    r.spawn_cap = x.spawn_cap;
    first = false;
    hipEvent_t ev;
    if (r.is_delete) {
      ev = T.begin(s, TK_DELETE);
      HIP_TRY(launch_plan_delete(t->g, r, s));
      T.end(TK_DELETE, ev, s);
    } else {
      // the fresh planner's wavefronts leave the evict list in regions
      ev = T.begin(s, TK_FRESH);
      HIP_TRY(launch_plan_fresh(t->g, r, s));
      T.end(TK_FRESH, ev, s);
      ev = T.begin(s, TK_EVICT);
      HIP_TRY(launch_plan_evict(t->g, r, t->evict_grid, s));
      T.end(TK_EVICT, ev, s);
    }
    ev = T.begin(s, TK_COMMIT);
    HIP_TRY(launch_commit(t->g, r, s));
    T.end(TK_COMMIT, ev, s);
    f.cur ^= 1;
  }
  // the statistics (gated on this list and the gate); their first kernel
  // writes the summary the host reads once this event has completed
  hipEvent_t ev = T.begin(s, TK_STATS);
  HIP_TRY(launch_batch_stats(r, f.m, f.slots, x.block_tmp, r.is_delete, c->cnt[f.cur], s));
  T.end(TK_STATS, ev, s);
  HIP_TRY(hipEventRecord(t->ctr_ready[f.set], s));
  return CK_OK;
}

// Waits for a sub-batch's counters; *done tells whether its last list came
// out empty (its statistics have then applied).
ck_status settle(ck_table* t, Flight& f, hipStream_t s, bool* done) {
  HIP_TRY(hipEventSynchronize(t->ctr_ready[f.set]));
  t->timer.collect();
  const HostSum& c = t->h_sum[f.set];
  if (c.overflow || c.overflow_seen) {  // a void round: a larger arena for what follows
    if (f.fixed) return CK_ENOMEM;     // fixed scratch never grows
    ck_status st = grow_arena(t);
    if (st != CK_OK) return st;
    // the flags are seen: clear them before any later round of this
    // sub-batch (the only user of this counter set until it is done) runs,
    // or each later look would grow the arena again
    HIP_TRY(hipMemsetAsync(&t->ctr[f.set].overflow, 0, 2 * sizeof(uint32_t), s));
  }
  *done = c.done != 0;
  if (*done) {
    const uint32_t hint = std::min(kMaxTailHint, std::max<uint32_t>(1, c.rounds));
    if (f.r.is_delete) {
      t->tail_hint_del = hint;
    } else if (f.r.upsert) {
      t->rounds += c.rounds;
      t->tail_prev_ups = t->tail_hint_ups;
      t->tail_hint_ups = hint;
    } else {
      t->rounds += c.rounds;
      t->tail_prev = t->tail_hint;
      t->tail_hint = hint;
    }
  }
  return CK_OK;
}

// Runs a sub-batch's remaining rounds until its last list is empty.
ck_status finish(ck_table* t, Flight& f, hipStream_t s) {
  for (;;) {
    bool done = false;
    ck_status st = settle(t, f, s, &done);
    if (st != CK_OK) return st;
    if (done) return CK_OK;
    st = enqueue_rounds(t, f, t->opt.enqueue_rounds ? t->opt.enqueue_rounds : 2, false, nullptr,
                        s);
    if (st != CK_OK) return st;
  }
}

ck_status run_batches(ck_table* t, const uint64_t* keys, const void* vals, uint64_t n,
                      uint8_t* status, uint32_t* views, uint32_t* kicks, uint32_t* retries,
                      bool is_delete, hipStream_t s, const uint32_t* op_table = nullptr,
                      const uint2* tdesc = nullptr, bool overwrite = false,
                      bool upsert = false, const Scratch* fixed = nullptr) {
  const uint32_t vb = t->B == 1 ? 4 : 8;
  const Scratch x = fixed ? *fixed : own_scratch(t);
  const uint64_t slots = t->bins * t->B;
  Flight prev;
  int set = 0;
  for (uint64_t b0 = 0; b0 < n; b0 += t->opt.batch_ops) {
    const uint64_t m = std::min<uint64_t>(t->opt.batch_ops, n - b0);
    uint32_t* ops[5] = {views ? views + b0 : x.op[0], x.op[1],
                        kicks ? kicks + b0 : x.op[2], retries ? retries + b0 : x.op[3],
                        x.op[4]};
    Flight f;
    f.fixed = fixed;
    f.r = make_round(t, x, keys + b0, vals ? (const char*)vals + b0 * vb : nullptr, status + b0, ops,
                     t->insert_count + b0, is_delete, op_table ? op_table + b0 : nullptr, tdesc);
    f.r.overwrite = overwrite ? 1u : 0u;
    f.r.upsert = upsert ? 1u : 0u;
    f.m = m;
    f.slots = op_table ? 0 : slots;  // density bands are per table: a group keeps totals only
    f.set = set;
    f.guard = 2 * m + 64;
    f.live = true;
    set ^= 1;
    const uint32_t K = t->opt.enqueue_rounds ? t->opt.enqueue_rounds
                       : is_delete           ? t->tail_hint_del + 1
                       : upsert              ? std::max(t->tail_hint_ups, t->tail_prev_ups)
                                             : std::max(t->tail_hint, t->tail_prev);
    const uint32_t* gate = prev.live ? &x.ctr[prev.set].unfinished : nullptr;
    ck_status st = enqueue_rounds(t, f, K, true, gate, s);
    if (st != CK_OK) return st;
    if (prev.live) {
      bool done = false;
      st = settle(t, prev, s, &done);
      if (st != CK_OK) return st;
      if (!done) {
        // this sub-batch saw a non-empty gate and did nothing: finish the
        // previous one, then enqueue this one again
        st = enqueue_rounds(t, prev, t->opt.enqueue_rounds ? t->opt.enqueue_rounds : 2, false,
                            nullptr, s);
        if (st == CK_OK) st = finish(t, prev, s);
        if (st == CK_OK) st = enqueue_rounds(t, f, K, true, nullptr, s);
        if (st != CK_OK) return st;
      }
    }
    prev = f;
  }
  if (prev.live) {
    ck_status st = finish(t, prev, s);
    if (st != CK_OK) return st;
  }
  if (!is_delete) t->insert_count += n;
  return CK_OK;
}

}  // namespace

extern "C" {

void ck_default_options(ck_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_chain = 500;
  o->max_search = 500;
  o->batch_ops = 1u << 20;
}

ck_status ck_storage_bytes(uint64_t bins, uint32_t B, uint32_t d, size_t* out) {
  if (!out || !geometry_ok(bins, B, d)) return CK_EINVAL;
  *out = layout(bins, B).total;
  return CK_OK;
}

static ck_status create_table(uint64_t bins, uint32_t B, uint32_t d, ck_scheme scheme,
                              const ck_options* opt, void* storage, size_t bytes, void* stream,
                              ck_table** out, uint32_t n_tables = 1);

ck_status ck_create(uint64_t bins, uint32_t B, uint32_t d, ck_scheme scheme,
                    const ck_options* opt, void* storage, size_t bytes, void* stream,
                    ck_table** out) {
  if (!out || !storage || !geometry_ok(bins, B, d)) return CK_EINVAL;
  return create_table(bins, B, d, scheme, opt, storage, bytes, stream, out);
}

static ck_status create_table(uint64_t bins, uint32_t B, uint32_t d, ck_scheme scheme,
                              const ck_options* opt, void* storage, size_t bytes, void* stream,
                              ck_table** out, uint32_t n_tables) {
  *out = nullptr;
  ck_options o;
  ck_default_options(&o);
  if (opt) o = *opt;
  if ((int)scheme < CK_RANDOM_WALK || (int)scheme > CK_HYBRID) return CK_EINVAL;
  if (scheme == CK_RATTLE && (B != 1 || o.ghost)) return CK_EINVAL;
  if (scheme == CK_QUEUE && d != 2) return CK_EINVAL;
  if (o.ghost && d != 2) return CK_EINVAL;
  if (o.load_balance && d != 2) return CK_EINVAL;
  if (o.batch_ops == 0 || o.batch_ops > (1u << 26)) return CK_EINVAL;
  if (o.max_chain > 2048 || o.max_search > 1024 || o.max_search < d) return CK_EINVAL;
  if (o.stash > kMaxStash) return CK_EINVAL;
  if (o.hash_bias > 4) return CK_EINVAL;
  if (o.spawn_k > 1) {  // k-at-a-time spawning: the group step of the two-choice searches
    if (scheme != CK_BFS && scheme != CK_SORTED) return CK_EUNSUPPORTED;
    if (d != 2 || (B != 4 && B != 8)) return CK_EUNSUPPORTED;
    if (o.spawn_k > 32 / B) return CK_EINVAL;
  }
  if (((uintptr_t)storage & 255) != 0) return CK_EINVAL;
  const Layout L = layout(bins, B);
  if (bytes < L.total) return CK_ENOMEM;
  ck_table* t = new (std::nothrow) ck_table();
  if (!t) return CK_ENOMEM;
  t->opt = o;
  t->bins = bins;
  t->B = B;
  t->H = d;
  t->scheme = scheme;
  uint64_t s = o.hash_seed;
  for (int i = 0; i < 4; ++i) {
    t->g.a[i] = sm_next(s) | 1ull;
    t->g.c[i] = sm_next(s);
  }
  char* base = (char*)storage;
  t->g.slots = (ulonglong2*)(base + L.slots);
  t->g.meta = (uint32_t*)(base + L.meta);
  t->g.owner = (unsigned long long*)(base + L.owner);
  t->g.n = (uint32_t)bins;
  t->g.B = B;
  t->g.H = d;
  t->g.scheme = scheme;
  t->g.ghost = o.ghost;
  t->g.balance = o.load_balance;
  t->g.max_chain = o.max_chain;
  t->g.max_search = o.max_search;
  t->g.rng_seed = o.rng_seed;
  t->g.stash_n = o.stash;
  t->g.hash_bias = o.hash_bias;
  t->g.spawn_k = o.spawn_k > 1 ? o.spawn_k : 0;
  t->g.stash_tables = n_tables;
  ck_status st = alloc_scratch(t);
  if (st != CK_OK) {
    free_scratch(t);
    delete t;
    return st;
  }
  if (launch_init(t->g, (hipStream_t)stream) != hipSuccess) {
    free_scratch(t);
    delete t;
    return CK_EDEVICE;
  }
  *out = t;
  return CK_OK;
}

static uint64_t sum_wg_views(ck_table* t, hipStream_t s, ck_status* st);

ck_status ck_clear(ck_table* t, void* stream) {
  if (!t) return CK_EINVAL;
  if (t->timer.on) {  // keep the timing's view count continuous across a clear
    ck_status st;
    const uint64_t cur = sum_wg_views(t, (hipStream_t)stream, &st);
    if (st != CK_OK) return st;
    t->timer.views_acc += cur - t->timer.views_base;
    t->timer.views_base = 0;
  }
  HIP_TRY(launch_init(t->g, (hipStream_t)stream));
  HIP_TRY(hipMemsetAsync(t->dstats, 0, sizeof(DevStats), (hipStream_t)stream));
  HIP_TRY(hipMemsetAsync(t->wg_views, 0, (size_t)t->evict_grid * 8, (hipStream_t)stream));
  t->insert_count = 0;
  t->rounds = 0;
  t->lookups = 0;
  return CK_OK;
}

ck_status ck_insert_ex(ck_table* t, const uint64_t* keys, const void* vals, uint64_t n,
                       uint8_t* status, uint32_t* views, uint32_t* kicks, uint32_t* retries,
                       void* stream) {
  if (!t) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!keys || !vals || !status) return CK_EINVAL;
  return run_batches(t, keys, vals, n, status, views, kicks, retries, false, (hipStream_t)stream);
}

ck_status ck_insert(ck_table* t, const uint64_t* keys, const void* vals, uint64_t n,
                    uint8_t* status, void* stream) {
  return ck_insert_ex(t, keys, vals, n, status, nullptr, nullptr, nullptr, stream);
}

ck_status ck_lookup_lpp(ck_table* t, const uint64_t* keys, uint64_t n, void* vals_out,
                        uint8_t* found, uint32_t lpp, void* stream) {
  if (!t) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!keys || !vals_out || !found) return CK_EINVAL;
  if (lpp == 0) lpp = t->B;
  if (lpp != 1 && lpp != t->B) return CK_EINVAL;
  hipEvent_t ev = t->timer.begin((hipStream_t)stream, TK_LOOKUP);
  HIP_TRY(launch_lookup(t->g, keys, n, vals_out, found, lpp, t->dstats, nullptr, nullptr,
                        (hipStream_t)stream));
  t->timer.end(TK_LOOKUP, ev, (hipStream_t)stream);
  t->lookups += n;
  return CK_OK;
}

ck_status ck_lookup(ck_table* t, const uint64_t* keys, uint64_t n, void* vals_out,
                    uint8_t* found, void* stream) {
  return ck_lookup_lpp(t, keys, n, vals_out, found, 0, stream);
}

ck_status ck_delete(ck_table* t, const uint64_t* keys, uint64_t n, uint8_t* found,
                    void* stream) {
  if (!t) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!keys || !found) return CK_EINVAL;
  return run_batches(t, keys, nullptr, n, found, nullptr, nullptr, nullptr, true,
                     (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The no-allocation delete: the round scratch of ck_delete carved from one
// fixed device array instead of the table's own scratch.
// ---------------------------------------------------------------------------
// Every GPU the library runs on holds its own copy of this array until the
// process ends.  Host code never passes the array's name to a kernel or a
// runtime call (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns, looked up once per device
// with that device current.
static __device__ __align__(256) unsigned char scratch[CK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The fixed array's device address on the current device (looked up on the
// first call there).
ck_status scratch_base(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CK_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return CK_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CK_OK;
}

// The delete path's round scratch for sub-batches of up to M ops, carved in
// 256-byte aligned pieces from `base` (or only sized, when base is null):
// two pending lists, plan headers, inline moves, five per-op counters, two
// round-counter sets and the statistics' staging.  Deletes write inline plans
// only, so no plan arena, spawn arena or evict list is carved.  Returns the
// bytes used.
size_t carve_delete_scratch(unsigned char* base, uint32_t M, Scratch* x) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)(base + off) : nullptr;
    off += align256(std::max<size_t>(bytes, 1));
    return p;
  };
  Scratch v{};
  v.stripe_cap = stripe_capacity(M);
  for (int k = 0; k < 2; ++k)
    v.pend[k] = (uint32_t*)take((size_t)kStripes * v.stripe_cap * sizeof(uint32_t));
  v.hdr = (uint4*)take((size_t)M * sizeof(uint4));
  v.hdr_spawn = (uint2*)take((size_t)M * sizeof(uint2));
  v.imv = (IMove*)take((size_t)M * kExtraInline * sizeof(IMove));
  for (int k = 0; k < 5; ++k) v.op[k] = (uint32_t*)take((size_t)M * sizeof(uint32_t));
  v.ctr = (Ctr*)take(2 * sizeof(Ctr));
  v.block_tmp = (uint32_t*)take(stats_tmp_words(M) * sizeof(uint32_t));
  v.evict = v.evict_cnt = v.spawns = nullptr;
  v.arena = nullptr;
  v.arena_cap = v.spawn_cap = 0;
  v.fixed = true;
  if (x) *x = v;
  return off;
}

}  // namespace

extern "C" {

ck_status ck_delete_noalloc(ck_table* t, const uint64_t* keys, uint64_t n, uint8_t* found,
                            void* stream) {
  static_assert(sizeof(scratch) == CK_NOALLOC_SCRATCH_BYTES, "scratch size");
  if (!t) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!keys || !found) return CK_EINVAL;
  // the largest sub-batch of this call must fit the fixed scratch
  if (std::min<uint64_t>(n, t->opt.batch_ops) > CK_NOALLOC_MAX_OPS) return CK_EINVAL;
  if (carve_delete_scratch(nullptr, CK_NOALLOC_MAX_OPS, nullptr) > CK_NOALLOC_SCRATCH_BYTES)
    return CK_EUNSUPPORTED;
  void* base = nullptr;
  ck_status st = scratch_base(&base);
  if (st != CK_OK) return st;
  Scratch x;
  carve_delete_scratch((unsigned char*)base, CK_NOALLOC_MAX_OPS, &x);
  hipStream_t s = (hipStream_t)stream;
  // the array keeps the last call's contents: the round counters start at
  // zero (cleared by a small fill kernel rather than a memset)
  HIP_TRY(launch_fill_u32((uint32_t*)x.ctr, 0u, 2 * sizeof(Ctr) / sizeof(uint32_t), s));
  // kernel-class timing creates events on demand: off for this call
  const bool timing = t->timer.on;
  t->timer.on = false;
  st = run_batches(t, keys, nullptr, n, found, nullptr, nullptr, nullptr, true, s, nullptr,
                   nullptr, false, false, &x);
  t->timer.on = timing;
  return st;
}

// Transactional batches (Sec. 8): per sub-batch of transactions, rounds of
// a planning launch and a commit launch, each one lane per pending
// transaction, until none is pending; the host reads the pending count
// after every round.
ck_status ck_transact(ck_table* t, const uint8_t* kind, const uint64_t* keys,
                      const uint64_t* vals, const uint32_t* off, uint32_t n_txn, uint8_t* status,
                      uint64_t* vals_out, uint32_t* txn_round, void* stream) {
  if (!t) return CK_EINVAL;
  if (n_txn == 0) return CK_OK;
  if (!kind || !keys || !vals || !off || !status || !vals_out || !txn_round) return CK_EINVAL;
  if ((t->scheme != CK_RANDOM_WALK && t->scheme != CK_QUEUE) || t->H != 2 ||
      (t->B != 2 && t->B != 4 && t->B != 8) || t->opt.ghost || t->g.stash_n || t->g.hash_bias ||
      t->g.stash_tables != 1)
    return CK_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  uint32_t ends[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&ends[0], off, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&ends[1], off + n_txn, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ends[1] < ends[0]) return CK_EINVAL;
  const uint32_t cap = std::min<uint32_t>(t->opt.batch_ops, 1u << 14);
  const size_t lane = txn_lane_bytes(t->g);
  if (t->txn_cap < cap) {
    (void)hipFree(t->txn_scratch);
    for (auto& l : t->txn_list) (void)hipFree(l);
    (void)hipFree(t->txn_nob);
    (void)hipFree(t->txn_lost);
    (void)hipFree(t->txn_cnt);
    t->txn_cap = 0;
    HIP_TRY(dalloc(&t->txn_scratch, (size_t)cap * lane));
    for (auto& l : t->txn_list) HIP_TRY(dalloc(&l, cap));
    HIP_TRY(dalloc(&t->txn_nob, cap));
    HIP_TRY(dalloc(&t->txn_lost, cap));
    HIP_TRY(dalloc(&t->txn_cnt, 1));
    t->txn_cap = cap;
  }
  const uint64_t op_base = t->insert_count;
  for (uint32_t t0 = 0; t0 < n_txn; t0 += cap) {
    const uint32_t m = std::min<uint32_t>(cap, n_txn - t0);
    HIP_TRY(launch_fill_u32(t->txn_lost, 0u, m, s));
    TxnRound r{};
    r.kind = kind;
    r.keys = keys;
    r.vals = vals;
    r.off = off;
    r.t0 = t0;
    r.pend = nullptr;  // round 0: every transaction of the sub-batch, in order
    r.npend = m;
    r.next_cnt = t->txn_cnt;
    r.status = status;
    r.vout = vals_out;
    r.txn_round = txn_round;
    r.lost = t->txn_lost;
    r.nob = t->txn_nob;
    r.max_rounds = t->opt.max_rounds;
    r.op_base = op_base;
    r.scratch = t->txn_scratch;
    r.lane_bytes = (uint32_t)lane;
    r.undo_cap = txn_undo_cap(t->g);
    r.stats = t->dstats;
    uint32_t round = 0;
    int cur = 0;
    while (r.npend) {
      // the smallest pending transaction commits or aborts every round
      if (round > m + 64) return CK_EDEVICE;
      ++t->epoch;
      if (t->epoch == 0) {  // claim tags wrapped: reset every claim word
        HIP_TRY(hipMemsetAsync(t->g.owner, 0xFF, (size_t)t->bins * 8, s));
        t->epoch = 1;
      }
      r.tag = (unsigned long long)(~t->epoch) << 32;
      r.round = round;
      r.next = t->txn_list[cur];
      HIP_TRY(launch_fill_u32(t->txn_cnt, 0u, 1, s));
      HIP_TRY(launch_txn(t->g, r, false, s));
      HIP_TRY(launch_txn(t->g, r, true, s));
      uint32_t n_next = 0;
      HIP_TRY(hipMemcpyAsync(&n_next, t->txn_cnt, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (n_next > r.npend) return CK_EDEVICE;
      r.pend = t->txn_list[cur];
      r.npend = n_next;
      cur ^= 1;
      ++round;
    }
    t->rounds += round;
  }
  t->insert_count += ends[1] - ends[0];
  return CK_OK;
}

ck_status ck_overwrite(ck_table* t, const uint64_t* keys, const void* vals, uint64_t n,
                       uint8_t* found, void* stream) {
  if (!t) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!keys || !vals || !found) return CK_EINVAL;
  return run_batches(t, keys, vals, n, found, nullptr, nullptr, nullptr, true,
                     (hipStream_t)stream, nullptr, nullptr, true);
}

ck_status ck_upsert(ck_table* t, const uint64_t* keys, const void* vals, uint64_t n,
                    uint8_t* status, uint32_t* views, uint32_t* kicks, uint32_t* retries,
                    void* stream) {
  if (!t) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!keys || !vals || !status) return CK_EINVAL;
  return run_batches(t, keys, vals, n, status, views, kicks, retries, false,
                     (hipStream_t)stream, nullptr, nullptr, false, true);
}

// The sum of the device accumulators' copies (the maximum for max_kicks).
static DevStatLine stats_sum(const DevStats& ds) {
  DevStatLine d;
  std::memset(&d, 0, sizeof(d));
  for (int k = 0; k < kStatStripes; ++k) {
    const DevStatLine& x = ds.s[k];
    for (int j = 0; j < S_NUM; ++j)
      d.v[j] = j == S_MAX_KICKS ? std::max(d.v[j], x.v[j]) : d.v[j] + x.v[j];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < CK_BANDS; ++b) d.band[a][b] += x.band[a][b];
  }
  return d;
}

ck_status ck_stats_get(ck_table* t, ck_stats* out, void* stream) {
  if (!t || !out) return CK_EINVAL;
  std::vector<DevStats> dv(1);
  HIP_TRY(hipMemcpyAsync(dv.data(), t->dstats, sizeof(DevStats), hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  const DevStatLine d = stats_sum(dv[0]);
  std::memset(out, 0, sizeof(*out));
  out->inserts_ok = d.v[S_INS_OK];
  out->inserts_failed = d.v[S_INS_FAIL];
  out->inserts_aborted = d.v[S_INS_ABORT];
  out->inserts_bad_key = d.v[S_INS_BAD];
  out->views = d.v[S_VIEWS];
  out->views_all = d.v[S_VIEWS_ALL];
  out->kicks = d.v[S_KICKS];
  out->max_kicks = d.v[S_MAX_KICKS];
  out->retries = d.v[S_RETRIES];
  out->rounds = t->rounds;
  out->twin_updates = d.v[S_TWINS];
  out->lookups = t->lookups;
  out->lookup_hits = d.v[S_LOOKUP_HITS];
  out->lookup_probes = d.v[S_LOOKUP_PROBES];
  out->deletes = d.v[S_DELETES];
  out->deletes_found = d.v[S_DEL_FOUND];
  out->delete_probes = d.v[S_DEL_PROBES];
  out->delete_retries = d.v[S_DEL_RETRIES];
  out->stored = d.v[S_STORED];
  for (int b = 0; b < CK_BANDS; ++b) {
    out->band_inserts[b] = d.band[0][b];
    out->band_views[b] = d.band[1][b];
    out->band_kicks[b] = d.band[2][b];
    out->band_fails[b] = d.band[3][b];
  }
  out->arena_moves = t->arena_cap;
  out->inserts_stashed = d.v[S_INS_STASHED];
  return CK_OK;
}

ck_status ck_stats_reset(ck_table* t, void* stream) {
  if (!t) return CK_EINVAL;
  std::vector<DevStats> dv(1);
  HIP_TRY(hipMemcpyAsync(dv.data(), t->dstats, sizeof(DevStats), hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  const unsigned long long stored = stats_sum(dv[0]).v[S_STORED];
  std::memset(dv.data(), 0, sizeof(DevStats));
  dv[0].s[0].v[S_STORED] = stored;
  HIP_TRY(hipMemcpyAsync(t->dstats, dv.data(), sizeof(DevStats), hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  t->rounds = 0;
  t->lookups = 0;
  return CK_OK;
}

static uint64_t sum_wg_views(ck_table* t, hipStream_t s, ck_status* st) {
  std::vector<unsigned long long> v(t->evict_grid);
  *st = CK_OK;
  if (hipMemcpyAsync(v.data(), t->wg_views, v.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    *st = CK_EDEVICE;
    return 0;
  }
  uint64_t sum = 0;
  for (auto x : v) sum += x;
  return sum;
}

ck_status ck_timing_enable(ck_table* t, uint32_t mask) {
  if (!t) return CK_EINVAL;
  HIP_TRY(hipDeviceSynchronize());
  t->timer.reset();
  t->timer.on = mask != 0;
  t->timer.mask = mask;
  ck_status st;
  t->timer.views_acc = 0;
  t->timer.views_base = sum_wg_views(t, nullptr, &st);
  return st;
}

ck_status ck_timing_get(ck_table* t, ck_timing* out, void* stream) {
  if (!t || !out) return CK_EINVAL;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  t->timer.collect();
  ck_kernel_time* dst[TK_N] = {&out->plan_fresh, &out->plan_evict, &out->plan_delete,
                               &out->commit,     &out->stats,      &out->lookup};
  for (int k = 0; k < TK_N; ++k) {
    dst[k]->launches = t->timer.launches[k];
    dst[k]->ms = t->timer.ms[k];
  }
  ck_status st;
  const uint64_t v = sum_wg_views(t, (hipStream_t)stream, &st);
  out->evict_views = t->timer.views_acc + v - t->timer.views_base;
  return st;
}

ck_status ck_export(ck_table* t, uint64_t* keys, uint64_t* vals, uint16_t* rattle,
                    uint32_t* meta, void* stream) {
  if (!t || !keys || !vals || !rattle || !meta) return CK_EINVAL;
  const uint64_t S = t->bins * t->B;
  std::vector<ulonglong2> buf(S);
  HIP_TRY(hipMemcpyAsync(buf.data(), t->g.slots, S * 16, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipMemcpyAsync(meta, t->g.meta, t->bins * 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  for (uint64_t i = 0; i < S; ++i) {
    keys[i] = buf[i].x;
    if (t->B == 1) {
      vals[i] = buf[i].y & 0xFFFFFFFFull;
      rattle[i] = (uint16_t)((buf[i].y >> 32) & 0xFFFF);
    } else {
      vals[i] = buf[i].y;
      rattle[i] = 0;
    }
  }
  return CK_OK;
}

ck_status ck_import(ck_table* t, const uint64_t* keys, const uint64_t* vals,
                    const uint16_t* rattle, const uint32_t* meta, void* stream) {
  if (!t || !keys || !vals || !rattle || !meta) return CK_EINVAL;
  const uint64_t S = t->bins * t->B;
  std::vector<ulonglong2> buf(S);
  uint64_t single = 0, dups = 0;
  for (uint64_t i = 0; i < S; ++i) {
    buf[i].x = keys[i];
    if (t->B == 1) buf[i].y = (vals[i] & 0xFFFFFFFFull) | ((uint64_t)rattle[i] << 32);
    else buf[i].y = vals[i];
    if (keys[i] != kEmpty) {
      if ((meta[i / t->B] >> (i % t->B)) & 1u) ++dups;
      else ++single;
    }
  }
  HIP_TRY(hipMemcpyAsync(t->g.slots, buf.data(), S * 16, hipMemcpyHostToDevice, (hipStream_t)stream));
  HIP_TRY(hipMemcpyAsync(t->g.meta, meta, t->bins * 4, hipMemcpyHostToDevice, (hipStream_t)stream));
  HIP_TRY(hipMemsetAsync(t->g.owner, 0xFF, t->bins * 8, (hipStream_t)stream));
  std::vector<ulonglong2> empty_stash;
  if (t->g.stash_n) {  // the image has no stash: emptied here, ck_import_stash fills it
    const size_t ns = (size_t)t->g.stash_tables * t->g.stash_n;
    empty_stash.assign(ns, make_ulonglong2(kEmpty, 0ull));
    HIP_TRY(hipMemcpyAsync(t->g.stash, empty_stash.data(), ns * 16, hipMemcpyHostToDevice,
                           (hipStream_t)stream));
    HIP_TRY(hipMemsetAsync(t->g.stash_owner, 0xFF, ns * 8, (hipStream_t)stream));
    HIP_TRY(hipMemsetAsync(t->g.stash_cnt, 0, (size_t)t->g.stash_tables * 4,
                           (hipStream_t)stream));
  }
  // the table's count goes to the first copy, the other copies' counts are zeroed
  const unsigned long long stored[2] = {single + dups / 2, 0};
  for (int k = 0; k < kStatStripes; ++k)
    HIP_TRY(hipMemcpyAsync(&t->dstats->s[k].v[S_STORED], &stored[k == 0 ? 0 : 1], 8,
                           hipMemcpyHostToDevice, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return CK_OK;
}

// Stash entries [first, first + stash_n) to or from host memory.
static ck_status stash_export(ck_table* t, uint32_t table, uint64_t* keys, uint64_t* vals,
                              void* stream) {
  const uint32_t S = t->g.stash_n;
  if (!S || !keys || !vals || table >= t->g.stash_tables) return CK_EINVAL;
  std::vector<ulonglong2> buf(S);
  HIP_TRY(hipMemcpyAsync(buf.data(), t->g.stash + (size_t)table * S, S * 16,
                         hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  for (uint32_t j = 0; j < S; ++j) {
    keys[j] = buf[j].x;
    vals[j] = buf[j].y;
  }
  return CK_OK;
}

ck_status ck_export_stash(ck_table* t, uint64_t* keys, uint64_t* vals, void* stream) {
  if (!t) return CK_EINVAL;
  return stash_export(t, 0, keys, vals, stream);
}

ck_status ck_import_stash(ck_table* t, const uint64_t* keys, const uint64_t* vals,
                          void* stream) {
  if (!t || !keys || !vals || !t->g.stash_n) return CK_EINVAL;
  const uint32_t S = t->g.stash_n;
  std::vector<ulonglong2> buf(S);
  uint32_t used = 0;
  for (uint32_t j = 0; j < S; ++j) {
    buf[j].x = keys[j];
    buf[j].y = t->B == 1 ? (vals[j] & 0xFFFFFFFFull) : vals[j];
    used += keys[j] != kEmpty;
  }
  std::vector<DevStats> dv(1);
  HIP_TRY(hipMemcpyAsync(dv.data(), t->dstats, sizeof(DevStats), hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  const unsigned long long stored = dv[0].s[0].v[S_STORED] + used;
  HIP_TRY(hipMemcpyAsync(t->g.stash, buf.data(), S * 16, hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  HIP_TRY(hipMemsetAsync(t->g.stash_owner, 0xFF, (size_t)S * 8, (hipStream_t)stream));
  HIP_TRY(hipMemcpyAsync(t->g.stash_cnt, &used, 4, hipMemcpyHostToDevice, (hipStream_t)stream));
  HIP_TRY(hipMemcpyAsync(&t->dstats->s[0].v[S_STORED], &stored, 8, hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return CK_OK;
}

ck_status ck_hash(const ck_table* t, uint64_t key, uint64_t* out) {
  if (!t || !out) return CK_EINVAL;
  for (uint32_t i = 0; i < t->H; ++i) {
    uint64_t z = t->g.a[i] * key + t->g.c[i];
    uint64_t b = (uint64_t)(((unsigned __int128)z * t->bins) >> 64);
    if (t->g.hash_bias) {  // as the kernels' hash_key
      uint64_t w = z;
      w = (w ^ (w >> 30)) * 0xBF58476D1CE4E5B9ull;
      w = (w ^ (w >> 27)) * 0x94D049BB133111EBull;
      w ^= w >> 31;
      if ((w & 3) < t->g.hash_bias)
        b = std::min<uint64_t>(b, (uint64_t)(((unsigned __int128)w * t->bins) >> 64));
    }
    for (;;) {
      bool clash = false;
      for (uint32_t j = 0; j < i; ++j) clash |= out[j] == b;
      if (!clash) break;
      b = (b + 1 == t->bins) ? 0 : b + 1;
    }
    out[i] = b;
  }
  return CK_OK;
}

uint64_t ck_insert_count(const ck_table* t) { return t ? t->insert_count : 0; }

ck_status ck_destroy(ck_table* t) {
  if (!t) return CK_EINVAL;
  (void)hipDeviceSynchronize();
  free_scratch(t);
  delete t;
  return CK_OK;
}

// ---------------------------------------------------------------------------
// groups: many tables of uneven sizes in one bin array, served by the same
// launches (every op carries its table index)
// ---------------------------------------------------------------------------
struct ck_group {
  ck_table* t = nullptr;
  std::vector<uint64_t> base, bins;
  uint2* d_tdesc = nullptr;
};

static bool group_geometry(uint32_t n_tables, const uint64_t* bins, uint32_t B, uint32_t d,
                           uint64_t* total) {
  if (n_tables == 0 || !bins) return false;
  uint64_t sum = 0;
  for (uint32_t i = 0; i < n_tables; ++i) {
    if (!geometry_ok(bins[i], B, d)) return false;
    sum += bins[i];
  }
  if (sum >= (1ull << 32)) return false;
  *total = sum;
  return true;
}

ck_status ck_group_storage_bytes(uint32_t n_tables, const uint64_t* bins, uint32_t B,
                                 uint32_t d, size_t* out) {
  uint64_t total = 0;
  if (!out || !group_geometry(n_tables, bins, B, d, &total)) return CK_EINVAL;
  *out = layout(total, B).total;
  return CK_OK;
}

ck_status ck_group_create(uint32_t n_tables, const uint64_t* bins, uint32_t B, uint32_t d,
                          ck_scheme scheme, const ck_options* opt, void* storage, size_t bytes,
                          void* stream, ck_group** out) {
  uint64_t total = 0;
  if (!out || !storage || !group_geometry(n_tables, bins, B, d, &total)) return CK_EINVAL;
  *out = nullptr;
  ck_group* G = new (std::nothrow) ck_group();
  if (!G) return CK_ENOMEM;
  ck_status st = create_table(total, B, d, scheme, opt, storage, bytes, stream, &G->t, n_tables);
  if (st != CK_OK) {
    delete G;
    return st;
  }
  std::vector<uint2> desc(n_tables);
  uint64_t b = 0;
  for (uint32_t i = 0; i < n_tables; ++i) {
    G->base.push_back(b);
    G->bins.push_back(bins[i]);
    desc[i] = make_uint2((uint32_t)b, (uint32_t)bins[i]);
    b += bins[i];
  }
  if (hipMalloc((void**)&G->d_tdesc, desc.size() * sizeof(uint2)) != hipSuccess ||
      hipMemcpy(G->d_tdesc, desc.data(), desc.size() * sizeof(uint2), hipMemcpyHostToDevice) !=
          hipSuccess) {
    ck_destroy(G->t);
    (void)hipFree(G->d_tdesc);
    delete G;
    return CK_EDEVICE;
  }
  *out = G;
  return CK_OK;
}

ck_status ck_group_insert(ck_group* G, const uint32_t* d_table, const uint64_t* keys,
                          const void* vals, uint64_t n, uint8_t* status, uint32_t* views,
                          uint32_t* kicks, uint32_t* retries, void* stream) {
  if (!G) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!d_table || !keys || !vals || !status) return CK_EINVAL;
  return run_batches(G->t, keys, vals, n, status, views, kicks, retries, false,
                     (hipStream_t)stream, d_table, G->d_tdesc);
}

ck_status ck_group_lookup(ck_group* G, const uint32_t* d_table, const uint64_t* keys, uint64_t n,
                          void* vals_out, uint8_t* found, uint32_t lpp, void* stream) {
  if (!G) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!d_table || !keys || !vals_out || !found) return CK_EINVAL;
  ck_table* t = G->t;
  if (lpp == 0) lpp = t->B;
  if (lpp != 1 && lpp != t->B) return CK_EINVAL;
  hipEvent_t ev = t->timer.begin((hipStream_t)stream, TK_LOOKUP);
  HIP_TRY(launch_lookup(t->g, keys, n, vals_out, found, lpp, t->dstats, d_table, G->d_tdesc,
                        (hipStream_t)stream));
  t->timer.end(TK_LOOKUP, ev, (hipStream_t)stream);
  t->lookups += n;
  return CK_OK;
}

ck_status ck_group_delete(ck_group* G, const uint32_t* d_table, const uint64_t* keys, uint64_t n,
                          uint8_t* found, void* stream) {
  if (!G) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!d_table || !keys || !found) return CK_EINVAL;
  return run_batches(G->t, keys, nullptr, n, found, nullptr, nullptr, nullptr, true,
                     (hipStream_t)stream, d_table, G->d_tdesc);
}

ck_status ck_group_overwrite(ck_group* G, const uint32_t* d_table, const uint64_t* keys,
                             const void* vals, uint64_t n, uint8_t* found, void* stream) {
  if (!G) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!d_table || !keys || !vals || !found) return CK_EINVAL;
  return run_batches(G->t, keys, vals, n, found, nullptr, nullptr, nullptr, true,
                     (hipStream_t)stream, d_table, G->d_tdesc, true);
}

ck_status ck_group_upsert(ck_group* G, const uint32_t* d_table, const uint64_t* keys,
                          const void* vals, uint64_t n, uint8_t* status, uint32_t* views,
                          uint32_t* kicks, uint32_t* retries, void* stream) {
  if (!G) return CK_EINVAL;
  if (n == 0) return CK_OK;
  if (!d_table || !keys || !vals || !status) return CK_EINVAL;
  return run_batches(G->t, keys, vals, n, status, views, kicks, retries, false,
                     (hipStream_t)stream, d_table, G->d_tdesc, false, true);
}

ck_status ck_group_export_stash(ck_group* G, uint32_t table, uint64_t* keys, uint64_t* vals,
                                void* stream) {
  if (!G) return CK_EINVAL;
  return stash_export(G->t, table, keys, vals, stream);
}

ck_status ck_group_export_table(ck_group* G, uint32_t table, uint64_t* keys, uint64_t* vals,
                                uint16_t* rattle, uint32_t* meta, void* stream) {
  if (!G || table >= G->bins.size() || !keys || !vals || !rattle || !meta) return CK_EINVAL;
  ck_table* t = G->t;
  const uint64_t b0 = G->base[table], nb = G->bins[table];
  const uint64_t S = nb * t->B;
  std::vector<ulonglong2> buf(S);
  HIP_TRY(hipMemcpyAsync(buf.data(), t->g.slots + b0 * t->B, S * 16, hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  HIP_TRY(hipMemcpyAsync(meta, t->g.meta + b0, nb * 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  for (uint64_t i = 0; i < S; ++i) {
    keys[i] = buf[i].x;
    vals[i] = t->B == 1 ? (buf[i].y & 0xFFFFFFFFull) : buf[i].y;
    rattle[i] = t->B == 1 ? (uint16_t)((buf[i].y >> 32) & 0xFFFF) : 0;
  }
  return CK_OK;
}

ck_status ck_group_stats_get(ck_group* G, ck_stats* out, void* stream) {
  if (!G) return CK_EINVAL;
  return ck_stats_get(G->t, out, stream);
}

ck_status ck_group_timing_enable(ck_group* G, uint32_t mask) {
  if (!G) return CK_EINVAL;
  return ck_timing_enable(G->t, mask);
}

ck_status ck_group_timing_get(ck_group* G, ck_timing* out, void* stream) {
  if (!G) return CK_EINVAL;
  return ck_timing_get(G->t, out, stream);
}

ck_status ck_group_clear(ck_group* G, void* stream) {
  if (!G) return CK_EINVAL;
  return ck_clear(G->t, stream);
}

uint64_t ck_group_insert_count(const ck_group* G) { return G ? G->t->insert_count : 0; }

ck_status ck_group_destroy(ck_group* G) {
  if (!G) return CK_EINVAL;
  ck_status st = ck_destroy(G->t);
  (void)hipFree(G->d_tdesc);
  delete G;
  return st;
}

const char* ck_strerror(ck_status s) {
  switch (s) {
    case CK_OK: return "ok";
    case CK_EINVAL: return "invalid argument";
    case CK_ENOMEM: return "out of memory or storage too small";
    case CK_EDEVICE: return "HIP runtime error";
    case CK_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

}  // extern "C"
