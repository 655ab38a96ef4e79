// ck_oracle.cpp -- reference model of a bucketized / d-ary cuckoo hash table
// with the kick-out eviction schemes of Kuszmaul, "Fast Concurrent Cuckoo
// Kick-out Eviction Schemes for High-Density Tables" (arXiv 1605.05236).
//
// TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU
// library is checked.  It is plain, single-threaded and deliberately slow:
// every algorithm is written as the paper states it, step by step, against a
// copy-on-write "draft" of the bins it touches.  It shares no code, header,
// constant table or helper with the GPU library, and the GPU library never
// calls it.  Only the tests, the smoke check and the CPU-baseline leg of the
// benchmark load it.
//
// Where the paper is silent or ambiguous the readings taken are listed in the
// repository's design notes; each is also stated next to the code below.
//
// Paper map:
//   Sec. 1  (Introduction)         two distinct bins per key, first-fit insert,
//                                  kick-out chains, constant-time lookup/delete.
//   Sec. 2  (Past work)            load balancing (insert into the less full bin);
//                                  stashing keys whose chains are abandoned.
//   Sec. 3  (Experimental setup)   uniformly random hashes; inserted keys are
//                                  assumed absent; cost = bins viewed per insert.
//   Sec. 4  (Ghost insertions)     duplicates in both bins; Proposition 4.1.
//   Sec. 5  (Sorted search)        BFS over records; spawn-count ordering with
//                                  16 buckets; visited-bin set; Theorem 5.1;
//                                  the sorted/BFS hybrid (depth, then count).
//   Sec. 6  (Queue-kicking)        FIFO victims via per-bin hit counters; hit
//                                  balancing; fetch-and-add slot scheduling.
//   Sec. 7  (Rattle-kicking)       d-ary tables, per-key rattle counters.
//   Sec. 8.2 (Mechanisms)          reverse-order ("system transaction") kick-out
//                                  chains; claims on every bin a plan writes.
//
// Parity status: every function here is pinned by the CPU tests (invariants,
// brute force, textbook dictionary semantics, closed forms and the paper's
// quoted statistics); see the test files for which pin covers which function.

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <vector>

namespace {

constexpr uint64_t kEmpty = ~0ull;  // reserved key marking an empty slot
constexpr int kBands = 200;         // 0.5 % density bands

enum Scheme { RANDOM_WALK = 0, BFS = 1, SORTED = 2, QUEUE = 3, RATTLE = 4, HYBRID = 5 };
enum OpStatus { ST_NOT_FOUND = 0, ST_OK = 1, ST_FAIL = 2, ST_ABORTED = 3, ST_BAD_KEY = 4,
                ST_UPDATED = 5, ST_STASHED = 6 };
constexpr uint32_t kMaxStash = 64;

// ---------------------------------------------------------------------------
// splitmix64 (Steele, Lea, Flood 2014): state advances by the golden-ratio
// increment and each output is the state passed through the mixing function.
// Used (a) to derive the hash multipliers from the hash seed and (b) as the
// counter-based generator behind the random walk's choices.
// ---------------------------------------------------------------------------
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t splitmix_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  return mix64(state);
}

// Uniform choice in [0, m) from a 64-bit word: floor(r * m / 2^64).
uint64_t scale(uint64_t r, uint64_t m) {
  return (uint64_t)(((unsigned __int128)r * m) >> 64);
}

struct Slot {
  uint64_t key = kEmpty;
  uint64_t val = 0;
  uint16_t rattle = 0;  // rattle counter r(x) of the stored key (Sec. 7)
};

// The state of one bin: its B slots plus the per-bin metadata the schemes
// keep: duplicate marks (Sec. 4), hit counter (Sec. 6), spawn count (Sec. 5).
struct BinState {
  Slot s[8];
  uint8_t dup = 0;  // bit i set: slot i holds a ghost duplicate
  uint8_t hc = 0;   // hit counter, one byte, wraps (Sec. 6 footnote)
  uint8_t sc = 0;   // spawn count, capped at 15 (four bits, Sec. 5)
};

struct Params {
  uint64_t n;        // bins
  int B;             // slots per bin
  int H;             // hash functions
  int scheme;
  int ghost;
  int load_balance;  // fresh insert into the less full bin (Sec. 2)
  uint32_t max_chain, max_search, max_rounds, batch_ops;
  uint64_t hash_seed, rng_seed;
  uint32_t stash = 0;  // stash entries (Sec. 2); 0: no stash
  uint32_t hash_bias = 0;  // 0: uniform hashes; 1-4: biased (Sec. 9)
  // BFS and sorted search spawning k records at a time (Sec. 5, Prefetching);
  // 0: the one-at-a-time searches
  uint32_t spawn_k = 0;
  // transactions: a plan that reads or writes more distinct bins than this
  // aborts (its claims and writes would not fit a bounded per-transaction
  // record)
  uint32_t txn_bins = 512;
};

struct Stats {
  uint64_t inserts_ok, inserts_failed, inserts_aborted, inserts_bad_key;
  uint64_t views, views_all, kicks, max_kicks, retries, rounds, twin_updates;
  uint64_t lookups, lookup_hits, lookup_probes;
  uint64_t deletes, deletes_found, delete_probes, delete_retries;
  uint64_t stored, inserts_stashed;
  uint64_t band_inserts[kBands], band_views[kBands], band_kicks[kBands], band_fails[kBands];
};

struct Table {
  Params p;
  uint64_t a[4], c[4];          // hash multipliers and offsets
  std::vector<BinState> bins;
  std::vector<Slot> stash;      // the stash (Sec. 2): key kEmpty marks a free entry
  uint64_t insert_count = 0;    // global index of the next insert op
  Stats st;
  // Optional record of every spawn-count increment (Sec. 5): the insert op
  // whose plan spawned a record, and the bin the record sat in.  Plans that
  // fail or lose a claim are recorded too, as their increments apply.
  bool log_spawns = false;
  std::vector<std::pair<uint64_t, uint64_t>> spawn_log;

  BinState bin(uint64_t b) const { return bins[b]; }

  // The stash entry holding key x, else -1; the first free entry, else -1.
  int stash_find(uint64_t x) const {
    for (size_t j = 0; j < stash.size(); ++j)
      if (stash[j].key == x) return (int)j;
    return -1;
  }
  int stash_free() const { return stash_find(kEmpty); }

  // Bin indices of key x (reading of Sec. 1 / Sec. 3): H distinct bins.
  // h_i(x) = floor(((a_i x + c_i) mod 2^64) * n / 2^64); a clash with an
  // earlier h_j is resolved by stepping to the next bin modulo n.
  //
  // Biased hashes (Sec. 9 asks how the schemes fare with them): with
  // hash_bias = k in 1..4, a second word w = mix64(z) decides by its two low
  // bits whether the choice is the lesser of floor(z n / 2^64) and
  // floor(w n / 2^64) (when they are below k, so for a fraction k / 4 of the
  // keys).  Bin b is then chosen with probability about
  //   (1 - k/4) / n + (k/4) (2 (n - b) - 1) / n^2,
  // from 1 + k/4 times the mean at bin 0 down to 1 - k/4 times it at the top.
  void hash(uint64_t x, uint64_t* out) const {
    for (int i = 0; i < p.H; ++i) {
      uint64_t z = a[i] * x + c[i];
      uint64_t h = scale(z, p.n);
      if (p.hash_bias) {
        const uint64_t w = mix64(z);
        if ((w & 3) < p.hash_bias) h = std::min(h, scale(w, p.n));
      }
      bool clash = true;
      while (clash) {
        clash = false;
        for (int j = 0; j < i; ++j)
          if (out[j] == h) clash = true;
        if (clash) h = (h + 1) % p.n;
      }
      out[i] = h;
    }
  }
};

// ---------------------------------------------------------------------------
// A plan: the algorithm run against a copy-on-write draft of the table.
// Reads see the draft where the plan has already written, else the table.
// The set of drafted bins is the plan's write set W (every bin whose slots,
// duplicate marks or hit counter the plan writes).  Spawn-count increments
// are collected separately: they are not writes to W (they are applied by
// every plan, including plans that fail or lose a claim).
// ---------------------------------------------------------------------------
struct Plan {
  const Table& T;
  uint64_t op;  // global insert index, keys the random choices
  uint32_t draws = 0;
  std::map<uint64_t, BinState> draft;
  std::set<uint64_t> claims;  // bins claimed without being written (upsert key claims)
  // At most one stash entry written: its index (-1: none) and new contents.
  int stash_at = -1;
  Slot stash_rec;
  std::vector<uint64_t> spawns;
  uint32_t views = 0, kicks = 0, twins = 0;
  int status = ST_FAIL;

  Plan(const Table& t, uint64_t op_) : T(t), op(op_) {}

  // Transactions (Sec. 8) record every bin whose contents a plan reads: its
  // read set, claimed like the write set.
  bool track_reads = false;
  mutable std::set<uint64_t> reads;

  BinState read(uint64_t b) const {
    if (track_reads) reads.insert(b);
    auto it = draft.find(b);
    return it != draft.end() ? it->second : T.bin(b);
  }
  BinState& write(uint64_t b) {
    auto it = draft.find(b);
    if (it == draft.end()) it = draft.emplace(b, T.bin(b)).first;
    return it->second;
  }
  // Reading a bin's slots to decide something: one bin viewed (Sec. 3).
  BinState view(uint64_t b) {
    ++views;
    return read(b);
  }

  // Counter-based random draw t of this plan: mix64(seed ^ op*phi ^ (t+1)).
  // A uniform choice among m > 1 options consumes one draw; m == 1 none.
  uint64_t uniform(uint64_t m) {
    if (m <= 1) return 0;
    uint64_t r = mix64(T.p.rng_seed ^ (op * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(draws + 1));
    ++draws;
    return scale(r, m);
  }

  int first_empty(const BinState& s) const {
    for (int i = 0; i < T.p.B; ++i)
      if (s.s[i].key == kEmpty) return i;
    return -1;
  }
  int first_dup(const BinState& s) const {
    for (int i = 0; i < T.p.B; ++i)
      if (s.s[i].key != kEmpty && ((s.dup >> i) & 1)) return i;
    return -1;
  }
  int occupancy(const BinState& s) const {
    int o = 0;
    for (int i = 0; i < T.p.B; ++i) o += s.s[i].key != kEmpty;
    return o;
  }
  // A bin ends a kick-out chain if it has a free slot, or, with ghost
  // insertions, a duplicate that can be dropped (Sec. 4).
  bool terminal(const BinState& s) const {
    return first_empty(s) >= 0 || (T.p.ghost && first_dup(s) >= 0);
  }

  // The key's bins other than `cur`, in hash order.
  std::vector<uint64_t> others(uint64_t key, uint64_t cur) const {
    uint64_t h[4];
    T.hash(key, h);
    std::vector<uint64_t> o;
    for (int i = 0; i < T.p.H; ++i)
      if (h[i] != cur) o.push_back(h[i]);
    return o;
  }

  // Store `rec` in slot i of bin b.  `as_dup` marks a ghost copy.  With the
  // queue scheme every insertion into a bin advances its hit counter (Sec. 6).
  void put(uint64_t b, int i, const Slot& rec, bool as_dup) {
    BinState& s = write(b);
    s.s[i] = rec;
    if (T.p.B == 1) s.s[i].val &= 0xFFFFFFFFull;  // single-slot bins keep 32-bit values
    if (as_dup) s.dup |= (uint8_t)(1u << i);
    else s.dup &= (uint8_t)~(1u << i);
    if (T.p.scheme == QUEUE) s.hc = (uint8_t)(s.hc + 1);
  }

  // Overwrite the duplicate in slot i of bin b: the other copy of that key,
  // in its other bin, stops being a duplicate (Sec. 4).  Reading the twin's
  // bin to find the copy is bookkeeping, not a bin viewed.
  void replace_dup(uint64_t b, int i, const Slot& rec) {
    uint64_t k = read(b).s[i].key;
    uint64_t tb = others(k, b)[0];
    BinState tw = read(tb);
    int ti = -1;
    for (int j = 0; j < T.p.B; ++j)
      if (tw.s[j].key == k) ti = j;
    write(tb).dup &= (uint8_t)~(1u << ti);
    ++twins;
    put(b, i, rec, false);
  }

  // Place `rec` into a terminal bin: a free slot first, else a duplicate.
  void place_terminal(uint64_t b, const Slot& rec) {
    BinState s = read(b);
    int e = first_empty(s);
    if (e >= 0) put(b, e, rec, false);
    else replace_dup(b, first_dup(s), rec);
  }

  // ---- The fresh insert, before any eviction (Sec. 1, 2, 4). -----------------
  // Returns true when the record was placed without a kick-out.
  bool place_fresh(const Slot& x, const uint64_t* h) {
    const Params& P = T.p;
    if (P.ghost) {
      // Ghost insertion (Sec. 4): both bins viewed; room in both -> a
      // duplicate copy in each; room in one -> there; else reuse a duplicate.
      BinState s0 = view(h[0]), s1 = view(h[1]);
      int e0 = first_empty(s0), e1 = first_empty(s1);
      if (e0 >= 0 && e1 >= 0) {
        put(h[0], e0, x, true);
        put(h[1], e1, x, true);
        return true;
      }
      if (e0 >= 0) { put(h[0], e0, x, false); return true; }
      if (e1 >= 0) { put(h[1], e1, x, false); return true; }
      int d0 = first_dup(s0);
      if (d0 >= 0) { replace_dup(h[0], d0, x); return true; }
      int d1 = first_dup(s1);
      if (d1 >= 0) { replace_dup(h[1], d1, x); return true; }
      return false;
    }
    if (P.load_balance || P.scheme == QUEUE) {
      // Load balancing (Sec. 2): view both, insert into the less full one.
      BinState s0 = view(h[0]), s1 = view(h[1]);
      int o0 = occupancy(s0), o1 = occupancy(s1);
      if (o0 < P.B || o1 < P.B) {
        uint64_t t = o0 <= o1 ? h[0] : h[1];
        put(t, first_empty(read(t)), x, false);
        return true;
      }
      return false;
    }
    // First fit (Sec. 1): look through the bins in hash order.
    for (int i = 0; i < P.H; ++i) {
      BinState s = view(h[i]);
      int e = first_empty(s);
      if (e >= 0) { put(h[i], e, x, false); return true; }
    }
    return false;
  }

  // ---- Random kicking (Sec. 1, Sec. 6 opening) --------------------------------
  void random_walk(const Slot& x, const uint64_t* h) {
    if (place_fresh(x, h)) { status = ST_OK; return; }
    uint64_t cur = h[uniform(T.p.H)];  // pick one of the key's bins
    Slot carry = x;
    for (;;) {
      if (kicks == T.p.max_chain) { status = ST_FAIL; return; }
      int i = (int)uniform(T.p.B);      // a random victim in it
      Slot victim = read(cur).s[i];
      put(cur, i, carry, false);
      ++kicks;
      carry = victim;
      std::vector<uint64_t> o = others(carry.key, cur);
      cur = o[uniform(o.size())];       // the victim goes to one of its other bins
      if (terminal(view(cur))) {
        place_terminal(cur, carry);
        status = ST_OK;
        return;
      }
    }
  }

  // ---- Queue-kicking with hit counters and hit balancing (Sec. 6) ---------------
  void queue_kick(const Slot& x, const uint64_t* h) {
    if (place_fresh(x, h)) { status = ST_OK; return; }
    // Both bins full: hit balancing picks the bin with the smaller counter.
    uint64_t t = read(h[0]).hc <= read(h[1]).hc ? h[0] : h[1];
    Slot carry = x;
    for (;;) {
      if (kicks == T.p.max_chain) { status = ST_FAIL; return; }
      // The record goes to slot (hit counter mod B), evicting the occupant;
      // with no deletes that occupant is the bin's oldest record.
      BinState s = read(t);
      int i = s.hc % T.p.B;
      Slot victim = s.s[i];
      put(t, i, carry, false);
      ++kicks;
      carry = victim;
      t = others(carry.key, t)[0];
      if (terminal(view(t))) {
        place_terminal(t, carry);
        status = ST_OK;
        return;
      }
    }
  }

  // ---- Breadth-first search, sorted search and their hybrid (Sec. 5) -------------
  // The search state is a list of records viewed but not yet spawned.  BFS
  // spawns them in FIFO order; sorted search spawns the one whose bin has the
  // smallest spawn count, kept as 16 FIFO buckets (bucket sort) keyed by the
  // capped spawn count read when the record enters the list.  The hybrid
  // orders first by the depth at which a record entered the search (the
  // records of the key's own bins have depth 0, those of a bin viewed while
  // spawning a depth-d record depth d + 1), then by that spawn count, FIFO
  // among equals.  Bins already visited by this search are never viewed
  // again, in all three.
  enum Order { BY_FIFO = 0, BY_COUNT = 1, BY_DEPTH_COUNT = 2 };
  struct Entry {
    uint64_t bin;
    int slot;
    int parent;  // index into `entries`, -1 for the records of the key's own bins
    int depth;
  };
  void search(const Slot& x, const uint64_t* h, Order order) {
    if (place_fresh(x, h)) { status = ST_OK; return; }
    std::vector<Entry> entries;
    // bucket[level][count]: level = depth for the hybrid, else 0
    std::vector<std::array<std::deque<int>, 16>> bucket(1);
    std::set<uint64_t> visited;
    auto enqueue_bin = [&](uint64_t b, int parent, int depth) {
      BinState s = read(b);
      int key = order != BY_FIFO ? std::min<int>(15, s.sc) : 0;
      size_t level = order == BY_DEPTH_COUNT ? (size_t)depth : 0;
      if (bucket.size() <= level) bucket.resize(level + 1);
      for (int i = 0; i < T.p.B; ++i) {
        entries.push_back({b, i, parent, depth});
        bucket[level][key].push_back((int)entries.size() - 1);
      }
    };
    for (int i = 0; i < T.p.H; ++i) {
      visited.insert(h[i]);
      enqueue_bin(h[i], -1, 0);
    }
    for (;;) {
      std::deque<int>* q = nullptr;
      for (size_t lv = 0; lv < bucket.size() && !q; ++lv)
        for (int k = 0; k < 16 && !q; ++k)
          if (!bucket[lv][k].empty()) q = &bucket[lv][k];
      if (!q) { status = ST_FAIL; return; }  // nothing left to spawn
      int e = q->front();
      q->pop_front();
      Entry en = entries[e];
      Slot rec = read(en.bin).s[en.slot];
      bool spawned = false;
      for (uint64_t child : others(rec.key, en.bin)) {
        if (visited.count(child)) continue;
        if (views == T.p.max_search) { status = ST_FAIL; return; }
        if (!spawned && order != BY_FIFO) spawns.push_back(en.bin);
        spawned = true;
        visited.insert(child);
        if (terminal(view(child))) {
          // Found: shift each record on the path one hop toward the free
          // slot, starting from the end of the chain (Sec. 8.2).
          place_terminal(child, rec);
          ++kicks;
          int cur = e;
          while (entries[cur].parent >= 0) {
            int par = entries[cur].parent;
            put(entries[cur].bin, entries[cur].slot, read(entries[par].bin).s[entries[par].slot], false);
            ++kicks;
            cur = par;
          }
          put(entries[cur].bin, entries[cur].slot, x, false);
          status = ST_OK;
          return;
        }
        enqueue_bin(child, e, en.depth + 1);
      }
    }
  }

  // ---- BFS and sorted search spawning k records at a time (Sec. 5) -------------
  // Sec. 5 (Prefetching) lets sorted search spawn the k records with the
  // smallest statistic at a time instead of one, so that their child bins can
  // be fetched together; BFS is the same with the FIFO order.  Reading taken:
  // the group is the first k records of the search order (across buckets);
  // their candidate bins not yet visited are viewed together, record by
  // record in group order, a view that would pass max_search ending the
  // viewing; every record that viewed a bin is spawned.  If a viewed bin ends
  // a chain, the first such bin in that order does (even when the cap cut the
  // group short); otherwise a capped group fails the search, and an uncapped
  // one lists every viewed bin as a new run, in that order.  With k = 1 this is
  // the one-at-a-time search whenever a record has a single candidate (two
  // hash functions).
  void search_k(const Slot& x, const uint64_t* h, Order order, uint32_t k) {
    if (place_fresh(x, h)) { status = ST_OK; return; }
    std::vector<Entry> entries;
    std::array<std::deque<int>, 16> bucket;  // FIFO per spawn count (BFS: one)
    std::set<uint64_t> visited;
    auto enqueue_bin = [&](uint64_t b, int parent, int depth) {
      BinState s = read(b);
      int key = order != BY_FIFO ? std::min<int>(15, s.sc) : 0;
      for (int i = 0; i < T.p.B; ++i) {
        entries.push_back({b, i, parent, depth});
        bucket[key].push_back((int)entries.size() - 1);
      }
    };
    for (int i = 0; i < T.p.H; ++i) {
      visited.insert(h[i]);
      enqueue_bin(h[i], -1, 0);
    }
    struct Viewed {
      int e;          // the record whose candidate it is
      uint64_t bin;
      bool term;
    };
    for (;;) {
      std::vector<int> group;
      for (int b = 0; b < 16 && group.size() < k; ++b)
        while (!bucket[b].empty() && group.size() < k) {
          group.push_back(bucket[b].front());
          bucket[b].pop_front();
        }
      if (group.empty()) { status = ST_FAIL; return; }  // nothing left to spawn
      std::vector<Viewed> seen;
      bool capped = false;
      for (int e : group) {
        const Entry en = entries[e];
        const Slot rec = read(en.bin).s[en.slot];
        bool spawned = false;
        for (uint64_t child : others(rec.key, en.bin)) {
          if (visited.count(child)) continue;
          if (views == T.p.max_search) { capped = true; break; }
          if (!spawned && order != BY_FIFO) spawns.push_back(en.bin);
          spawned = true;
          visited.insert(child);
          seen.push_back({e, child, terminal(view(child))});
        }
        if (capped) break;
      }
      for (const Viewed& v : seen) {
        if (!v.term) continue;
        // Found: the record moves into the terminal bin, each record on its
        // path moves one hop toward it, from the chain's end back (Sec. 8.2).
        place_terminal(v.bin, read(entries[v.e].bin).s[entries[v.e].slot]);
        ++kicks;
        int cur = v.e;
        while (entries[cur].parent >= 0) {
          int par = entries[cur].parent;
          put(entries[cur].bin, entries[cur].slot, read(entries[par].bin).s[entries[par].slot],
              false);
          ++kicks;
          cur = par;
        }
        put(entries[cur].bin, entries[cur].slot, x, false);
        status = ST_OK;
        return;
      }
      if (capped) { status = ST_FAIL; return; }
      for (const Viewed& v : seen) enqueue_bin(v.bin, v.e, entries[v.e].depth + 1);
    }
  }

  // ---- Rattle-kicking for d-ary tables with single-slot bins (Sec. 7) -----------
  // A key x carries a counter r(x), incremented on every try; it tries bin
  // h_{r mod d}.  Against an occupant y the larger counter keeps the bin (the
  // occupant on a tie) and the other key moves on.
  void rattle(const Slot& x, const uint64_t* h) {
    (void)h;
    Slot carry = x;
    carry.rattle = 0;
    uint32_t tries = 0;
    for (;;) {
      if (tries == T.p.max_chain) { status = ST_FAIL; return; }
      uint64_t hh[4];
      T.hash(carry.key, hh);
      uint64_t b = hh[carry.rattle % T.p.H];
      carry.rattle = (uint16_t)(carry.rattle + 1);
      ++tries;
      BinState s = view(b);
      if (s.s[0].key == kEmpty) {
        put(b, 0, carry, false);
        status = ST_OK;
        return;
      }
      Slot y = s.s[0];
      if (carry.rattle > y.rattle) {
        put(b, 0, carry, false);
        ++kicks;
        carry = y;
      }
    }
  }
};

Plan plan_insert(const Table& T, uint64_t op, uint64_t key, uint64_t val) {
  Plan pl(T, op);
  Slot x;
  x.key = key;
  x.val = val;
  uint64_t h[4];
  T.hash(key, h);
  switch (T.p.scheme) {
    case RANDOM_WALK: pl.random_walk(x, h); break;
    case BFS:
      if (T.p.spawn_k) pl.search_k(x, h, Plan::BY_FIFO, T.p.spawn_k);
      else pl.search(x, h, Plan::BY_FIFO);
      break;
    case SORTED:
      if (T.p.spawn_k) pl.search_k(x, h, Plan::BY_COUNT, T.p.spawn_k);
      else pl.search(x, h, Plan::BY_COUNT);
      break;
    case HYBRID: pl.search(x, h, Plan::BY_DEPTH_COUNT); break;
    case QUEUE: pl.queue_kick(x, h); break;
    case RATTLE: pl.rattle(x, h); break;
  }
  if (pl.status != ST_OK) {  // a failed plan writes nothing (table unchanged)
    pl.draft.clear();
    pl.kicks = 0;
    pl.twins = 0;
    // Stashing (Sec. 2): the key whose kick-out chain was abandoned goes to
    // the first free stash entry, if there is one.  Plans leave the table as
    // it was, so the homeless key is the inserted one.
    const int j = T.stash_free();
    if (j >= 0) {
      pl.status = ST_STASHED;
      pl.stash_at = j;
      pl.stash_rec.key = key;
      pl.stash_rec.val = T.p.B == 1 ? (val & 0xFFFFFFFFull) : val;
    }
  }
  return pl;
}

// Delete (Sec. 1): find the key in its bins and empty every slot holding it,
// both copies of a ghost duplicate included.  Counters are left unchanged.
Plan plan_delete(const Table& T, uint64_t key, uint32_t* probes) {
  Plan pl(T, 0);
  uint64_t h[4];
  T.hash(key, h);
  pl.status = ST_NOT_FOUND;
  *probes = 0;
  for (int i = 0; i < T.p.H; ++i) {
    BinState s = pl.read(h[i]);
    ++*probes;
    for (int j = 0; j < T.p.B; ++j) {
      if (s.s[j].key != key) continue;
      bool was_dup = (s.dup >> j) & 1;
      BinState& w = pl.write(h[i]);
      w.s[j] = Slot();
      w.dup &= (uint8_t)~(1u << j);
      if (was_dup) {
        uint64_t tb = h[1 - i];
        BinState t = pl.read(tb);
        ++*probes;
        for (int k = 0; k < T.p.B; ++k)
          if (t.s[k].key == key) {
            BinState& tw = pl.write(tb);
            tw.s[k] = Slot();
            tw.dup &= (uint8_t)~(1u << k);
          }
      }
      pl.status = ST_OK;
      return pl;
    }
  }
  if (!T.stash.empty()) {  // then the stash, searched as one unit
    ++*probes;
    const int j = T.stash_find(key);
    if (j >= 0) {
      pl.stash_at = j;
      pl.stash_rec = Slot();
      pl.status = ST_OK;
    }
  }
  return pl;
}

// Overwrite (Sec. 1): a stored key gets a new value in place, in every slot
// holding it (both copies of a ghost duplicate).  The key, its duplicate mark,
// its rattle counter and the bin's counters stay as they are.  An absent key
// is not found and changes nothing.
Plan plan_overwrite(const Table& T, uint64_t key, uint64_t val, uint32_t* probes) {
  Plan pl(T, 0);
  uint64_t h[4];
  T.hash(key, h);
  pl.status = ST_NOT_FOUND;
  *probes = 0;
  const uint64_t v = T.p.B == 1 ? (val & 0xFFFFFFFFull) : val;  // single-slot bins: 32-bit values
  for (int i = 0; i < T.p.H; ++i) {
    BinState s = pl.read(h[i]);
    ++*probes;
    for (int j = 0; j < T.p.B; ++j) {
      if (s.s[j].key != key) continue;
      bool was_dup = (s.dup >> j) & 1;
      pl.write(h[i]).s[j].val = v;
      if (was_dup) {
        uint64_t tb = h[1 - i];
        BinState t = pl.read(tb);
        ++*probes;
        for (int k = 0; k < T.p.B; ++k)
          if (t.s[k].key == key) pl.write(tb).s[k].val = v;
      }
      pl.status = ST_OK;
      return pl;
    }
  }
  if (!T.stash.empty()) {
    ++*probes;
    const int j = T.stash_find(key);
    if (j >= 0) {
      pl.stash_at = j;
      pl.stash_rec = T.stash[j];
      pl.stash_rec.val = v;
      pl.status = ST_OK;
    }
  }
  return pl;
}

// Upsert: a stored key gets the new value in place, as an overwrite (status
// UPDATED); an absent key is inserted with the table's scheme.  The presence
// check views the key's bins in hash order until the key turns up (all d of
// them when it is absent; reading a ghost twin is bookkeeping), and an
// absent key's plan adds its own views.  An absent key's plan also claims
// the key's first bin without writing it, so two upserts of one new key in a
// round conflict: the later one, next round, finds the key and overwrites it.
// With a stash, the stash is searched after the bins, as one more view.
Plan plan_upsert(const Table& T, uint64_t op, uint64_t key, uint64_t val) {
  uint64_t h[4];
  T.hash(key, h);
  uint32_t seen = 0;
  bool found = false;
  for (int i = 0; i < T.p.H && !found; ++i) {
    const BinState& s = T.bins[h[i]];
    ++seen;
    for (int j = 0; j < T.p.B; ++j)
      if (s.s[j].key == key) found = true;
  }
  if (!found && !T.stash.empty()) {
    ++seen;
    found = T.stash_find(key) >= 0;
  }
  if (found) {
    uint32_t probes = 0;
    Plan pl = plan_overwrite(T, key, val, &probes);
    pl.status = ST_UPDATED;
    pl.views = seen;
    return pl;
  }
  Plan pl = plan_insert(T, op, key, val);
  pl.views += seen;
  pl.claims.insert(h[0]);
  return pl;
}

// ---- Transactions (Sec. 8) --------------------------------------------------------
// A transaction is a run of operations -- lookups, inserts, deletes and
// overwrites -- applied atomically.  Reading taken (the round form of Sec. 8's
// plan / lock-and-verify / apply stages): in a round every pending
// transaction plans all its operations in order against the round-start
// snapshot, each one seeing the writes of the earlier ones (the plan's draft,
// which plays the part of Stage 1's deferred edits).  An insert runs the
// table's scheme whole, kick-out chain included, inside that draft; an insert
// whose chain fails leaves the draft as it was before it.  The transaction's
// read set (every bin whose contents it read: probes, views, the bins of its
// chains) and write set (every bin it writes) are both claimed with its index,
// the lowest index winning a bin, as claim flags do; a transaction that owns
// every bin of both sets commits all its writes, the others plan again next
// round (whole), and max_rounds turns a persistent loser into an abort.
// Winners' read and write sets are pairwise disjoint, so the committed
// transactions are equivalent to running them one at a time, round by round
// and within a round in index order: the table is transactional in Sec. 8's
// sense.  The random walk's choices of an insert are keyed by the insert's
// index in the call's operations.
enum TxnOp { TX_LOOKUP = 0, TX_INSERT = 1, TX_DELETE = 2, TX_OVERWRITE = 3 };

struct TxnResult {
  std::vector<uint8_t> status;  // per op of the transaction
  std::vector<uint64_t> value;  // lookups that hit
};

// Find key x through the plan's draft: (bin, slot) or bin kEmpty.
static std::pair<uint64_t, int> txn_find(Plan& pl, uint64_t x, const uint64_t* h) {
  for (int i = 0; i < pl.T.p.H; ++i) {
    BinState s = pl.read(h[i]);
    for (int j = 0; j < pl.T.p.B; ++j)
      if (s.s[j].key == x) return {h[i], j};
  }
  return {kEmpty, -1};
}

Plan plan_txn(const Table& T, const uint8_t* kind, const uint64_t* keys, const uint64_t* vals,
              uint64_t o0, uint64_t o1, uint64_t op_base, TxnResult* out) {
  Plan pl(T, 0);
  pl.track_reads = true;
  out->status.assign(o1 - o0, ST_NOT_FOUND);
  out->value.assign(o1 - o0, 0);
  for (uint64_t j = o0; j < o1; ++j) {
    const uint64_t x = keys[j];
    uint8_t& st = out->status[j - o0];
    if (x == kEmpty) { st = ST_BAD_KEY; continue; }
    uint64_t h[4];
    T.hash(x, h);
    if (kind[j] == TX_LOOKUP) {
      auto f = txn_find(pl, x, h);
      if (f.second >= 0) {
        st = ST_OK;
        out->value[j - o0] = pl.read(f.first).s[f.second].val;
      }
    } else if (kind[j] == TX_DELETE) {
      auto f = txn_find(pl, x, h);
      if (f.second >= 0) {
        BinState& w = pl.write(f.first);
        w.s[f.second] = Slot();
        w.dup &= (uint8_t)~(1u << f.second);
        st = ST_OK;
      }
    } else if (kind[j] == TX_OVERWRITE) {
      auto f = txn_find(pl, x, h);
      if (f.second >= 0) {
        pl.write(f.first).s[f.second].val = T.p.B == 1 ? (vals[j] & 0xFFFFFFFFull) : vals[j];
        st = ST_OK;
      }
    } else {  // insert (the key is assumed absent, Sec. 3)
      const auto saved = pl.draft;
      pl.op = op_base + j;
      pl.draws = 0;
      pl.kicks = 0;  // the chain and search caps are per insert
      pl.views = 0;
      pl.status = ST_FAIL;
      Slot r;
      r.key = x;
      r.val = vals[j];
      switch (T.p.scheme) {
        case RANDOM_WALK: pl.random_walk(r, h); break;
        case BFS: pl.search(r, h, Plan::BY_FIFO); break;
        case SORTED: pl.search(r, h, Plan::BY_COUNT); break;
        case HYBRID: pl.search(r, h, Plan::BY_DEPTH_COUNT); break;
        case QUEUE: pl.queue_kick(r, h); break;
        case RATTLE: pl.rattle(r, h); break;
      }
      st = (uint8_t)pl.status;
      if (pl.status != ST_OK) pl.draft = saved;  // a failed insert writes nothing
    }
  }
  return pl;
}

// ---- Deterministic phased rounds ------------------------------------------------
// Every pending op plans against the same snapshot; each plan claims the bins
// it writes, lowest op index winning a bin; a plan that owns all its bins is
// applied (its writes land on exactly the contents it read), the others try
// again next round.  Spawn-count increments of all plans are added with
// saturation at 15 after each round.  A sub-batch of one op is the serial
// algorithm.
struct OpResult {
  int status = ST_FAIL;
  uint32_t views = 0, kicks = 0, twins = 0, retries = 0, views_all = 0;
};

template <class PlanFn>
uint32_t run_rounds(Table& T, const std::vector<uint64_t>& ids, PlanFn plan_fn,
                    std::vector<OpResult>& res) {
  std::vector<uint64_t> pending = ids;  // batch-relative op indices in op order
  uint32_t round = 0;
  while (!pending.empty()) {
    std::vector<Plan> plans;
    plans.reserve(pending.size());
    for (uint64_t i : pending) plans.push_back(plan_fn(i));
    // Claims: the lowest op index that writes (or claims) a bin owns it this
    // round.
    std::map<uint64_t, uint64_t> owner;
    auto take = [&](uint64_t b, uint64_t i) {
      auto it = owner.find(b);
      if (it == owner.end() || i < it->second) owner[b] = i;
    };
    for (size_t k = 0; k < plans.size(); ++k) {
      for (auto& kv : plans[k].draft) take(kv.first, pending[k]);
      for (uint64_t b : plans[k].claims) take(b, pending[k]);
      // stash entry j is claimed like one more bin, numbered n + j
      if (plans[k].stash_at >= 0) take(T.p.n + (uint64_t)plans[k].stash_at, pending[k]);
    }
    std::vector<uint64_t> next;
    for (size_t k = 0; k < plans.size(); ++k) {
      uint64_t i = pending[k];
      bool wins = true;
      for (auto& kv : plans[k].draft)
        if (owner[kv.first] != i) wins = false;
      for (uint64_t b : plans[k].claims)
        if (owner[b] != i) wins = false;
      if (plans[k].stash_at >= 0 && owner[T.p.n + (uint64_t)plans[k].stash_at] != i)
        wins = false;
      res[i].views_all += plans[k].views;
      if (wins) {
        for (auto& kv : plans[k].draft) {
          BinState nb = kv.second;
          nb.sc = T.bins[kv.first].sc;  // spawn counts are merged below
          T.bins[kv.first] = nb;
        }
        if (plans[k].stash_at >= 0) T.stash[(size_t)plans[k].stash_at] = plans[k].stash_rec;
        res[i].status = plans[k].status;
        res[i].views = plans[k].views;
        res[i].kicks = plans[k].kicks;
        res[i].twins = plans[k].twins;
      } else {
        ++res[i].retries;
        if (T.p.max_rounds && res[i].retries >= T.p.max_rounds) res[i].status = ST_ABORTED;
        else next.push_back(i);
      }
    }
    for (auto& pl : plans)
      for (uint64_t b : pl.spawns) {
        T.bins[b].sc = (uint8_t)std::min(15, T.bins[b].sc + 1);
        if (T.log_spawns) T.spawn_log.push_back({pl.op, b});
      }
    ++round;
    pending.swap(next);
  }
  return round;
}

}  // namespace

// ============================================================================
// C interface for the test harness (ctypes).
// ============================================================================
extern "C" {

struct ck_oracle_stats_t {
  uint64_t inserts_ok, inserts_failed, inserts_aborted, inserts_bad_key;
  uint64_t views, views_all, kicks, max_kicks, retries, rounds, twin_updates;
  uint64_t lookups, lookup_hits, lookup_probes;
  uint64_t deletes, deletes_found, delete_probes, delete_retries;
  uint64_t stored, inserts_stashed;
  uint64_t band_inserts[kBands], band_views[kBands], band_kicks[kBands], band_fails[kBands];
};

void* ck_oracle_create(uint64_t n, int B, int H, int scheme, int ghost, int load_balance,
                       uint32_t max_chain, uint32_t max_search, uint32_t max_rounds,
                       uint32_t batch_ops, uint64_t hash_seed, uint64_t rng_seed) {
  if (n < (uint64_t)H || B < 1 || B > 8 || H < 2 || H > 4 || batch_ops == 0) return nullptr;
  if (scheme < RANDOM_WALK || scheme > HYBRID) return nullptr;
  if (H > 2 && B != 1) return nullptr;                 // d-ary tables use single-slot bins
  if (ghost && H != 2) return nullptr;                 // ghosts need exactly two bins
  if (scheme == RATTLE && (B != 1 || ghost)) return nullptr;
  if (scheme == QUEUE && H != 2) return nullptr;
  if (load_balance && H != 2) return nullptr;           // balancing compares two bins
  Table* T = new Table();
  T->p = Params{n, B, H, scheme, ghost, load_balance, max_chain, max_search, max_rounds,
                batch_ops, hash_seed, rng_seed};
  uint64_t s = hash_seed;
  for (int i = 0; i < 4; ++i) {
    T->a[i] = splitmix_next(s) | 1ull;
    T->c[i] = splitmix_next(s);
  }
  T->bins.assign(n, BinState());
  std::memset(&T->st, 0, sizeof(T->st));
  return T;
}

void ck_oracle_destroy(void* t) { delete (Table*)t; }

// Start (on != 0) or stop recording spawn-count increments; starting clears
// the record.
void ck_oracle_log_spawns(void* tp, int on) {
  Table& T = *(Table*)tp;
  T.log_spawns = on != 0;
  if (T.log_spawns) T.spawn_log.clear();
}

// The recorded increments in the order they were applied: (insert op index,
// bin) pairs, at most `cap` of them copied.  Returns how many were recorded.
uint64_t ck_oracle_spawn_log(void* tp, uint64_t* ops, uint64_t* bins, uint64_t cap) {
  Table& T = *(Table*)tp;
  for (uint64_t k = 0; k < T.spawn_log.size() && k < cap; ++k) {
    ops[k] = T.spawn_log[k].first;
    bins[k] = T.spawn_log[k].second;
  }
  return T.spawn_log.size();
}

// Biased hashing of level k (0: uniform, up to 4), set on an empty table.
int ck_oracle_set_hash_bias(void* tp, uint32_t k) {
  Table& T = *(Table*)tp;
  if (k > 4) return -1;
  T.p.hash_bias = k;
  return 0;
}

// BFS or sorted search spawning k records at a time (k >= 1; 0 restores the
// one-at-a-time search), set on an empty table.
int ck_oracle_set_spawn_k(void* tp, uint32_t k) {
  Table& T = *(Table*)tp;
  if (T.p.scheme != BFS && T.p.scheme != SORTED) return -1;
  if (k > 64) return -1;
  T.p.spawn_k = k;
  return 0;
}

// The bound on the distinct bins one transaction's plan may touch (>= 1).
int ck_oracle_set_txn_bins(void* tp, uint32_t bins) {
  Table& T = *(Table*)tp;
  if (bins == 0) return -1;
  T.p.txn_bins = bins;
  return 0;
}

// Give an empty table a stash of `entries` entries (at most kMaxStash).
int ck_oracle_set_stash(void* tp, uint32_t entries) {
  Table& T = *(Table*)tp;
  if (entries > kMaxStash) return -1;
  T.p.stash = entries;
  T.stash.assign(entries, Slot());
  return 0;
}

// The stash's keys and values, entry by entry (key kEmpty: free).
void ck_oracle_export_stash(void* tp, uint64_t* keys, uint64_t* vals) {
  Table& T = *(Table*)tp;
  for (size_t j = 0; j < T.stash.size(); ++j) {
    keys[j] = T.stash[j].key;
    vals[j] = T.stash[j].val;
  }
}

// Load the stash (after ck_oracle_import, which counts the bins' keys).
void ck_oracle_import_stash(void* tp, const uint64_t* keys, const uint64_t* vals) {
  Table& T = *(Table*)tp;
  for (size_t j = 0; j < T.stash.size(); ++j) {
    T.stash[j].key = keys[j];
    T.stash[j].val = vals[j];
    T.stash[j].rattle = 0;
    if (keys[j] != kEmpty) ++T.st.stored;
  }
}

void ck_oracle_hash(void* t, uint64_t key, uint64_t* out) { ((Table*)t)->hash(key, out); }

// Insert n keys (assumed absent, Sec. 3).  Per-op outputs: status, bins
// viewed by the plan that decided the op, kicks, and rounds lost to claims.
// `op_ids` (may be null) gives each op's index for the walk's random choices;
// by default it is the table's running insert count.
static void insert_batch(void* tp, const uint64_t* keys, const uint64_t* vals,
                         const uint64_t* op_ids, uint64_t n, uint8_t* status, uint32_t* views,
                         uint32_t* kicks, uint32_t* retries, bool upsert) {
  Table& T = *(Table*)tp;
  const uint64_t slots = T.p.n * (uint64_t)T.p.B;
  for (uint64_t b0 = 0; b0 < n; b0 += T.p.batch_ops) {
    uint64_t m = std::min<uint64_t>(T.p.batch_ops, n - b0);
    uint64_t base = T.insert_count + b0;
    std::vector<uint64_t> ids;
    std::vector<OpResult> res(m);
    for (uint64_t i = 0; i < m; ++i) {
      if (keys[b0 + i] == kEmpty) res[i].status = ST_BAD_KEY;
      else ids.push_back(i);
    }
    auto fn = [&](uint64_t i) {
      const uint64_t op = op_ids ? op_ids[b0 + i] : base + i;
      return upsert ? plan_upsert(T, op, keys[b0 + i], vals[b0 + i])
                    : plan_insert(T, op, keys[b0 + i], vals[b0 + i]);
    };
    T.st.rounds += run_rounds(T, ids, fn, res);
    // Per-op results and density bands: an op's density is that of the table
    // had the sub-batch been applied one op at a time in op order.
    uint64_t ok_before = 0;
    for (uint64_t i = 0; i < m; ++i) {
      const OpResult& r = res[i];
      status[b0 + i] = (uint8_t)r.status;
      views[b0 + i] = r.status == ST_ABORTED ? 0 : r.views;
      kicks[b0 + i] = r.status == ST_OK ? r.kicks : 0;
      retries[b0 + i] = r.retries;
      if (r.status == ST_BAD_KEY) { ++T.st.inserts_bad_key; continue; }
      if (r.status == ST_UPDATED) continue;  // an upsert that overwrote: not an insert
      T.st.retries += r.retries;
      T.st.views_all += r.views_all;
      if (r.status == ST_ABORTED) { ++T.st.inserts_aborted; continue; }
      uint64_t band = (uint64_t)kBands * (T.st.stored + ok_before) / slots;
      if (band >= (uint64_t)kBands) band = kBands - 1;
      T.st.band_inserts[band] += 1;
      T.st.band_views[band] += r.views;
      T.st.views += r.views;
      if (r.status == ST_OK) {
        ++ok_before;
        ++T.st.inserts_ok;
        T.st.band_kicks[band] += r.kicks;
        T.st.kicks += r.kicks;
        T.st.max_kicks = std::max<uint64_t>(T.st.max_kicks, r.kicks);
        T.st.twin_updates += r.twins;
      } else {
        // the chain failed; a stashed key is still held by the table, and
        // `stored` counts every key held, in bins or in the stash
        if (r.status == ST_STASHED) {
          ++ok_before;
          ++T.st.inserts_stashed;
        } else {
          ++T.st.inserts_failed;
        }
        T.st.band_fails[band] += 1;
      }
    }
    T.st.stored += ok_before;
  }
  T.insert_count += n;
}

void ck_oracle_insert_ids(void* tp, const uint64_t* keys, const uint64_t* vals,
                          const uint64_t* op_ids, uint64_t n, uint8_t* status, uint32_t* views,
                          uint32_t* kicks, uint32_t* retries) {
  insert_batch(tp, keys, vals, op_ids, n, status, views, kicks, retries, false);
}

void ck_oracle_insert(void* tp, const uint64_t* keys, const uint64_t* vals, uint64_t n,
                      uint8_t* status, uint32_t* views, uint32_t* kicks, uint32_t* retries) {
  insert_batch(tp, keys, vals, nullptr, n, status, views, kicks, retries, false);
}

// Upsert n keys: stored keys get new values (status UPDATED), the others are
// inserted; per-op outputs as for inserts.
void ck_oracle_upsert(void* tp, const uint64_t* keys, const uint64_t* vals, uint64_t n,
                      uint8_t* status, uint32_t* views, uint32_t* kicks, uint32_t* retries) {
  insert_batch(tp, keys, vals, nullptr, n, status, views, kicks, retries, true);
}

void ck_oracle_upsert_ids(void* tp, const uint64_t* keys, const uint64_t* vals,
                          const uint64_t* op_ids, uint64_t n, uint8_t* status, uint32_t* views,
                          uint32_t* kicks, uint32_t* retries) {
  insert_batch(tp, keys, vals, op_ids, n, status, views, kicks, retries, true);
}

// Lookup (Sec. 1): the key is in one of its bins, probed in hash order.
void ck_oracle_lookup(void* tp, const uint64_t* keys, uint64_t n, uint64_t* vals_out,
                      uint8_t* found) {
  Table& T = *(Table*)tp;
  for (uint64_t q = 0; q < n; ++q) {
    uint64_t h[4];
    T.hash(keys[q], h);
    found[q] = 0;
    vals_out[q] = 0;
    ++T.st.lookups;
    if (keys[q] == kEmpty) continue;
    for (int i = 0; i < T.p.H && !found[q]; ++i) {
      ++T.st.lookup_probes;
      const BinState& s = T.bins[h[i]];
      for (int j = 0; j < T.p.B; ++j)
        if (s.s[j].key == keys[q]) {
          found[q] = 1;
          vals_out[q] = s.s[j].val;
          break;
        }
    }
    if (!found[q] && !T.stash.empty()) {  // then the stash, one more probe
      ++T.st.lookup_probes;
      const int j = T.stash_find(keys[q]);
      if (j >= 0) {
        found[q] = 1;
        vals_out[q] = T.stash[(size_t)j].val;
      }
    }
    T.st.lookup_hits += found[q];
  }
}

void ck_oracle_delete(void* tp, const uint64_t* keys, uint64_t n, uint8_t* found,
                      uint32_t* retries) {
  Table& T = *(Table*)tp;
  for (uint64_t b0 = 0; b0 < n; b0 += T.p.batch_ops) {
    uint64_t m = std::min<uint64_t>(T.p.batch_ops, n - b0);
    std::vector<uint64_t> ids;
    std::vector<OpResult> res(m);
    std::vector<uint32_t> probes(m, 0);
    for (uint64_t i = 0; i < m; ++i) {
      if (keys[b0 + i] == kEmpty) res[i].status = ST_BAD_KEY;
      else ids.push_back(i);
    }
    auto fn = [&](uint64_t i) { return plan_delete(T, keys[b0 + i], &probes[i]); };
    run_rounds(T, ids, fn, res);
    for (uint64_t i = 0; i < m; ++i) {
      found[b0 + i] = (uint8_t)res[i].status;
      retries[b0 + i] = res[i].retries;
      if (res[i].status == ST_BAD_KEY) continue;
      ++T.st.deletes;
      T.st.delete_retries += res[i].retries;
      T.st.delete_probes += probes[i];
      if (res[i].status == ST_OK) { ++T.st.deletes_found; --T.st.stored; }
    }
  }
}

// Overwrite n keys' values (a key absent is reported, nothing changes).
// Per-op outputs: status (found or not) and rounds lost to claims.  The
// table's counters are not changed.
void ck_oracle_overwrite(void* tp, const uint64_t* keys, const uint64_t* vals, uint64_t n,
                         uint8_t* found, uint32_t* retries) {
  Table& T = *(Table*)tp;
  for (uint64_t b0 = 0; b0 < n; b0 += T.p.batch_ops) {
    uint64_t m = std::min<uint64_t>(T.p.batch_ops, n - b0);
    std::vector<uint64_t> ids;
    std::vector<OpResult> res(m);
    std::vector<uint32_t> probes(m, 0);
    for (uint64_t i = 0; i < m; ++i) {
      if (keys[b0 + i] == kEmpty) res[i].status = ST_BAD_KEY;
      else ids.push_back(i);
    }
    auto fn = [&](uint64_t i) {
      return plan_overwrite(T, keys[b0 + i], vals[b0 + i], &probes[i]);
    };
    run_rounds(T, ids, fn, res);
    for (uint64_t i = 0; i < m; ++i) {
      found[b0 + i] = (uint8_t)res[i].status;
      retries[b0 + i] = res[i].retries;
    }
  }
}

// Transactional batch (Sec. 8): n_txn transactions, transaction t being the
// operations [txn_off[t], txn_off[t + 1]) of kind / keys / vals (kinds: 0
// lookup, 1 insert, 2 delete, 3 overwrite), applied in sub-batches of
// batch_ops transactions by the transaction rounds above.  Per op: status
// (lookup / delete / overwrite: found or not; insert: OK or FAIL; ABORTED for
// every op of an aborted transaction; BAD_KEY) and the value of a lookup
// that hit.  Per transaction: the round (within its sub-batch, from 0) in
// which it committed, and the rounds it lost.  Tables with ghosts or a stash
// are refused (-1); so are upserts, by having no kind for them.
int ck_oracle_txn(void* tp, const uint8_t* kind, const uint64_t* keys, const uint64_t* vals,
                  const uint64_t* txn_off, uint64_t n_txn, uint8_t* status, uint64_t* vals_out,
                  uint32_t* txn_round, uint32_t* txn_retries) {
  Table& T = *(Table*)tp;
  if (T.p.ghost || !T.stash.empty()) return -1;
  const uint64_t op_base = T.insert_count;
  for (uint64_t t0 = 0; t0 < n_txn; t0 += T.p.batch_ops) {
    const uint64_t m = std::min<uint64_t>(T.p.batch_ops, n_txn - t0);
    std::vector<uint64_t> pending;
    for (uint64_t i = 0; i < m; ++i) pending.push_back(i);
    std::vector<uint32_t> retries(m, 0);
    uint32_t round = 0;
    while (!pending.empty()) {
      std::vector<Plan> plans;
      std::vector<TxnResult> outs(pending.size());
      plans.reserve(pending.size());
      for (size_t k = 0; k < pending.size(); ++k) {
        const uint64_t t = t0 + pending[k];
        plans.push_back(plan_txn(T, kind, keys, vals, txn_off[t], txn_off[t + 1], op_base,
                                 &outs[k]));
      }
      std::map<uint64_t, uint64_t> owner;  // bin -> lowest transaction claiming it
      auto take = [&](uint64_t b, uint64_t i) {
        auto it = owner.find(b);
        if (it == owner.end() || i < it->second) owner[b] = i;
      };
      // a plan that touched more than txn_bins distinct bins aborts: no claims
      std::vector<bool> too_big(plans.size(), false);
      for (size_t k = 0; k < plans.size(); ++k) {
        std::set<uint64_t> touched(plans[k].reads);
        for (auto& kv : plans[k].draft) touched.insert(kv.first);
        too_big[k] = touched.size() > T.p.txn_bins;
      }
      for (size_t k = 0; k < plans.size(); ++k) {
        if (too_big[k]) continue;
        for (auto& kv : plans[k].draft) take(kv.first, pending[k]);
        for (uint64_t b : plans[k].reads) take(b, pending[k]);
      }
      std::vector<uint64_t> next;
      for (size_t k = 0; k < plans.size(); ++k) {
        const uint64_t i = pending[k], t = t0 + i;
        bool wins = !too_big[k];
        for (auto& kv : plans[k].draft)
          if (owner[kv.first] != i) wins = false;
        for (uint64_t b : plans[k].reads)
          if (owner[b] != i) wins = false;
        const uint64_t o0 = txn_off[t], o1 = txn_off[t + 1];
        if (wins) {
          for (auto& kv : plans[k].draft) {
            BinState nb = kv.second;
            nb.sc = T.bins[kv.first].sc;  // spawn counts are merged below
            T.bins[kv.first] = nb;
          }
          for (uint64_t j = o0; j < o1; ++j) {
            status[j] = outs[k].status[j - o0];
            vals_out[j] = outs[k].value[j - o0];
            if (status[j] == ST_OK && kind[j] == TX_INSERT) { ++T.st.stored; ++T.st.inserts_ok; }
            if (status[j] == ST_FAIL) ++T.st.inserts_failed;
            if (status[j] == ST_OK && kind[j] == TX_DELETE) { --T.st.stored; ++T.st.deletes_found; }
          }
          txn_round[t] = round;
          txn_retries[t] = retries[i];
        } else if (too_big[k] || (T.p.max_rounds && ++retries[i] >= T.p.max_rounds)) {
          for (uint64_t j = o0; j < o1; ++j) {
            status[j] = ST_ABORTED;
            vals_out[j] = 0;
          }
          txn_round[t] = round;
          txn_retries[t] = retries[i];
        } else {
          if (!T.p.max_rounds) ++retries[i];
          next.push_back(i);
        }
      }
      for (auto& pl : plans)
        for (uint64_t b : pl.spawns) {
          T.bins[b].sc = (uint8_t)std::min(15, T.bins[b].sc + 1);
          if (T.log_spawns) T.spawn_log.push_back({pl.op, b});
        }
      ++round;
      pending.swap(next);
    }
    T.st.rounds += round;
  }
  T.insert_count += txn_off[n_txn] - txn_off[0];
  return 0;
}

// Canonical image of the table: keys and values per slot, rattle counters
// per slot, and per bin the metadata word
//   bits 0-7 duplicate marks, bits 8-11 spawn count, bits 24-31 hit counter.
void ck_oracle_export(void* tp, uint64_t* keys, uint64_t* vals, uint16_t* rattle,
                      uint32_t* meta) {
  Table& T = *(Table*)tp;
  for (uint64_t b = 0; b < T.p.n; ++b) {
    const BinState& s = T.bins[b];
    for (int j = 0; j < T.p.B; ++j) {
      keys[b * T.p.B + j] = s.s[j].key;
      vals[b * T.p.B + j] = s.s[j].val;
      rattle[b * T.p.B + j] = s.s[j].rattle;
    }
    meta[b] = (uint32_t)s.dup | ((uint32_t)s.sc << 8) | ((uint32_t)s.hc << 24);
  }
}

// Load a canonical image (inverse of export); `stored` is recomputed.
void ck_oracle_import(void* tp, const uint64_t* keys, const uint64_t* vals,
                      const uint16_t* rattle, const uint32_t* meta) {
  Table& T = *(Table*)tp;
  uint64_t distinct = 0;
  for (uint64_t b = 0; b < T.p.n; ++b) {
    BinState& s = T.bins[b];
    for (int j = 0; j < T.p.B; ++j) {
      s.s[j].key = keys[b * T.p.B + j];
      s.s[j].val = vals[b * T.p.B + j];
      s.s[j].rattle = rattle[b * T.p.B + j];
      if (s.s[j].key != kEmpty && !((meta[b] >> j) & 1)) ++distinct;
    }
    s.dup = (uint8_t)(meta[b] & 0xFF);
    s.sc = (uint8_t)((meta[b] >> 8) & 0xF);
    s.hc = (uint8_t)(meta[b] >> 24);
  }
  // Every ghost pair contributes two duplicate-marked copies of one key.
  uint64_t dups = 0;
  for (uint64_t b = 0; b < T.p.n; ++b)
    for (int j = 0; j < T.p.B; ++j)
      if (T.bins[b].s[j].key != kEmpty && ((T.bins[b].dup >> j) & 1)) ++dups;
  T.st.stored = distinct + dups / 2;
}

static_assert(sizeof(ck_oracle_stats_t) == sizeof(Stats), "the C view of the counters");

void ck_oracle_stats(void* tp, ck_oracle_stats_t* out) {
  std::memcpy(out, &((Table*)tp)->st, sizeof(ck_oracle_stats_t));
}

uint64_t ck_oracle_insert_count(void* tp) { return ((Table*)tp)->insert_count; }

}  // extern "C"
