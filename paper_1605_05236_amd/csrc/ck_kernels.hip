// ck_kernels.hip -- gfx950 kernels of libck.
//
// Kernel map (one sub-batch of inserts runs plan -> commit rounds):
//   k_init          empty table (keys all-ones, metadata zero, claims reset)
//   k_lookup        lane group of LPP lanes per query; each probe loads one
//                   bin as one coalesced 64/128-byte access and ballots for the
//                   key (Sec. 1: the key is in one of its bins)
//   k_plan_fresh    lane group of B/2 lanes per pending insert: views the
//                   key's bins and plans the placement when no kick-out is
//                   needed (first fit, load balancing, ghost insertion,
//                   duplicate reuse); an upsert first looks for its key and,
//                   if stored, plans the new value; every other op goes to its
//                   wavefront's region of the evict list for an eviction planner
//   k_plan_walk     eight walks per wavefront: random kicking, queue-kicking,
//                   rattle-kicking; the chain is logged (LDS, then scratch)
//                   and later bin reads see the chain's own earlier writes
//   k_plan_search   four searches per wavefront: BFS, sorted search and their
//                   hybrid over runs of B records, several frontier bins per
//                   load
//   k_plan_delete   lane group per pending delete or overwrite
//   k_commit        2 lanes per plan: claim check, reverse-order chain write,
//                   metadata atomics, spawn-count updates; the losers form
//                   the next round's pending list
//   k_stats_*       per-op counters -> totals and density bands
//
// Every planner reads the round-start snapshot only and claims each bin it
// will write with a 64-bit atomicMin on the bin's claim word.  A failed insert
// plan may claim a stash entry instead (Sec. 2).  The round kernels and the
// lookup come in a plain instance and an extended one (upserts, a stash,
// biased hashes).
#include <hip/hip_runtime.h>

#include "ck_internal.h"

namespace ck {

// ---------------------------------------------------------------------------
// hashing and randomness
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// h_i(x) = floor(((a_i x + c_i) mod 2^64) * n / 2^64), stepped past clashes,
// in the bin range [t.base, t.base + t.n) of the key's table (a group of
// tables shares one bin array; a single table has base 0).  A biased hash of
// level k (Sec. 9's open question) takes the lesser of that bin and the bin
// of w = mix64(a_i x + c_i) when the two low bits of w are below k, so low
// bins are favoured for a fraction k / 4 of the keys.
// (Kernels instantiated for uniform hashes pass MayBias = false, which drops
// the biased branch and its registers.)
template <int H, bool MayBias = true>
__device__ __forceinline__ void hash_key(const Geo& g, Tab t, uint64_t x, uint32_t* h) {
  const uint32_t end = t.base + t.n;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const uint64_t z = g.a[i] * x + g.c[i];
    uint32_t b = t.base + (uint32_t)__umul64hi(z, (uint64_t)t.n);
    if (MayBias && g.hash_bias) {
      const uint64_t w = mix64(z);
      if ((uint32_t)(w & 3) < g.hash_bias)
        b = min(b, t.base + (uint32_t)__umul64hi(w, (uint64_t)t.n));
    }
    for (;;) {
      bool clash = false;
#pragma unroll
      for (int j = 0; j < i; ++j) clash |= (h[j] == b);
      if (!clash) break;
      b = (b + 1 == end) ? t.base : b + 1;
    }
    h[i] = b;
  }
}

// True when the pending list with segment counts `cnt` is not empty (all 64
// lanes call it together).
__device__ __forceinline__ bool list_open(const uint32_t* cnt) {
  const uint32_t c = cnt[(threadIdx.x & 63) * kStripeWords];
  return __ballot(c != 0) != 0ull;
}

// The round's pending list as one wavefront sees it.  The first round of a
// sub-batch lists every op in order (position = op index, count a kernel
// argument); later rounds read the segment counts the previous commit left
// (lane l loads segment l's count) and map a position to its segment through
// their prefix sums.  A round whose gate (the previous sub-batch's last
// list) is not empty sees no ops.  init and at are called by all 64 lanes
// together.
struct Pending {
  const uint32_t* list = nullptr;
  uint32_t cap = 0, n = 0, incl = 0, excl = 0;
  bool ident = true;
  __device__ void init(const Round& r) {
    ident = r.first != 0;
    if (r.gate && *r.gate) {  // the previous sub-batch is not finished
      ident = true;
      n = 0;
      return;
    }
    if (ident) {
      n = r.npend;
      return;
    }
    list = r.pend;
    cap = r.stripe_cap;
    const int lane = threadIdx.x & 63;
    const uint32_t c = r.pcnt[lane * kStripeWords];
    uint32_t x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    incl = x;
    excl = x - c;
    n = __shfl(x, 63, 64);
  }
  // op index at position p, kNone for p >= n
  __device__ uint32_t at(uint32_t p) const {
    if (ident) return p < n ? p : kNone;
    // segment of p: the number of segments whose inclusive prefix is <= p
    uint32_t sg = 0;
#pragma unroll
    for (uint32_t step = 32; step; step >>= 1)
      if (__shfl(incl, (int)(sg + step - 1), 64) <= p) sg += step;
    const uint32_t e = __shfl(excl, (int)(sg & 63), 64);
    if (p >= n) return kNone;
    return list[(size_t)sg * cap + (p - e)];
  }
};

// The table of op i: from the group's descriptors, else the single table.
__device__ __forceinline__ Tab tab_of(const Geo& g, const uint32_t* op_table, const uint2* tdesc,
                                      uint64_t i) {
  if (op_table) {
    const uint2 d = tdesc[op_table[i]];
    return Tab{d.x, d.y};
  }
  return Tab{0u, g.n};
}

// ---------------------------------------------------------------------------
// the stash (Sec. 2): stash_n entries per table, searched after the bins
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t table_of(const uint32_t* op_table, uint64_t i) {
  return op_table ? op_table[i] : 0u;
}

// The entry of table t's stash that holds key x (not the empty key), or
// kNone.  A group of W lanes searches it together: lane gl reads entries
// gl, gl + W, ...; `vote` gives the group's ballot, bit k for its lane k.
template <class Vote>
__device__ __forceinline__ uint32_t stash_find(const Geo& g, uint32_t t, uint64_t x, int gl,
                                               int W, Vote vote) {
  if (g.stash_cnt[t] == 0) return kNone;
  const uint32_t sb = t * g.stash_n;
  for (uint32_t c = 0; c < g.stash_n; c += (uint32_t)W) {
    const uint64_t k = c + gl < g.stash_n ? g.stash[sb + c + gl].x : kEmpty;
    const uint64_t m = vote(k == x);
    if (m) return sb + c + (uint32_t)(__ffsll((unsigned long long)m) - 1);
  }
  return kNone;
}

// Uniform choice in [0, m): draw t of op `op`; m == 1 consumes no draw.
__device__ __forceinline__ uint32_t uniform_choice(const Geo& g, uint64_t op, uint32_t& draws,
                                                   uint32_t m) {
  if (m <= 1) return 0;
  uint64_t r = mix64(g.rng_seed ^ (op * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(draws + 1));
  ++draws;
  return (uint32_t)__umul64hi(r, (uint64_t)m);
}

__device__ __forceinline__ uint64_t load_aux(const void* vals, uint32_t i, int B) {
  if (B == 1) return (uint64_t)((const uint32_t*)vals)[i];
  return ((const uint64_t*)vals)[i];
}

__device__ __forceinline__ uint32_t ffs32(uint32_t m) { return (uint32_t)(__ffs(m) - 1); }

__device__ __forceinline__ uint32_t rattle_of(uint64_t aux) { return (uint32_t)((aux >> 32) & 0xFFFF); }
__device__ __forceinline__ uint64_t with_rattle(uint64_t aux, uint32_t r) {
  return (aux & 0xFFFFFFFFull) | ((uint64_t)(r & 0xFFFF) << 32);
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint64_t count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = value;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, value, (uint64_t)count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
__global__ void k_init(Geo g) {
  const uint64_t nslots = (uint64_t)g.n * g.B;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += stride)
    g.slots[i] = make_ulonglong2(kEmpty, 0ull);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += stride) {
    g.meta[i] = 0u;
    g.owner[i] = ~0ull;
  }
  const uint64_t nstash = (uint64_t)g.stash_tables * g.stash_n;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nstash; i += stride) {
    g.stash[i] = make_ulonglong2(kEmpty, 0ull);
    g.stash_owner[i] = ~0ull;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
       i < (nstash ? g.stash_tables : 0u); i += stride)
    g.stash_cnt[i] = 0u;
}

hipError_t launch_init(const Geo& g, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(2048), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// block reduction helper (u64 sum over a block of up to 1024 threads)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Block-wide sum of two counters, one atomic per block and counter.
__device__ __forceinline__ void block_add2(unsigned long long a, unsigned long long b,
                                           unsigned long long* da, unsigned long long* db) {
  __shared__ unsigned long long s_acc[2];
  if (threadIdx.x == 0) { s_acc[0] = 0; s_acc[1] = 0; }
  __syncthreads();
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    if (a) atomicAdd(&s_acc[0], a);
    if (b) atomicAdd(&s_acc[1], b);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_acc[0]) atomicAdd(da, s_acc[0]);
    if (s_acc[1]) atomicAdd(db, s_acc[1]);
  }
}

// ---------------------------------------------------------------------------
// lookup: LPP lanes per query, B/LPP slots per lane
// ---------------------------------------------------------------------------
// EXT: the instance for tables with a stash or biased hashes.
// A lane group takes QL queries per pass (two where a lane holds at most two
// slots of a bin): their keys, hashes and probes of the same hash function
// are issued together, so twice the line loads are in flight per wavefront
// for the same bytes (the second probe is still issued only for a query the
// first did not answer).
template <int B, int LPP>
__host__ __device__ constexpr int lookup_queries_per_group() {
  return B / LPP <= 2 ? 2 : 1;
}
template <int B, int LPP, int H, bool EXT>
__global__ __launch_bounds__(256) void k_lookup(Geo g, const uint64_t* __restrict__ keys,
                                                uint64_t n, void* __restrict__ out,
                                                uint8_t* __restrict__ found, DevStats* st,
                                                const uint32_t* op_table, const uint2* tdesc) {
  constexpr int SPL = B / LPP;
  constexpr int QL = lookup_queries_per_group<B, LPP>();
  constexpr int GPB = 256 / LPP;   // lane groups per block
  constexpr int QPB = GPB * QL;    // queries per block and pass
  const int lane = threadIdx.x & 63;
  const int gl = lane % LPP;
  const int gshift = lane - gl;
  const uint64_t gmask = (LPP == 64) ? ~0ull : ((1ull << LPP) - 1);
  unsigned long long probes_acc = 0, hits_acc = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * QPB; base < n;
       base += (uint64_t)gridDim.x * QPB) {
    // query u of this group: base + u GPB + group index (each u a coalesced run)
    uint64_t qv[QL], x[QL], val[QL];
    bool active[QL], hit[QL];
    uint32_t probes[QL], h[QL][H];
    int winner[QL];
#pragma unroll
    for (int u = 0; u < QL; ++u) {
      qv[u] = base + (uint64_t)u * GPB + threadIdx.x / LPP;
      active[u] = qv[u] < n;
      x[u] = active[u] ? keys[qv[u]] : kEmpty;
      probes[u] = 0;
      hit[u] = false;
      val[u] = 0;
      winner[u] = 0;
    }
#pragma unroll
    for (int u = 0; u < QL; ++u) {
#pragma unroll
      for (int hi = 0; hi < H; ++hi) h[u][hi] = 0;
      if (x[u] != kEmpty) hash_key<H, EXT>(g, tab_of(g, op_table, tdesc, qv[u]), x[u], h[u]);
    }
#pragma unroll
    for (int hi = 0; hi < H; ++hi) {
      // the probes of hash function hi of every query not yet answered
      bool want[QL];
      ulonglong2 sl[QL][SPL];
#pragma unroll
      for (int u = 0; u < QL; ++u) {
        want[u] = x[u] != kEmpty && !hit[u];
        if (want[u]) {
          const ulonglong2* p = g.slots + (uint64_t)h[u][hi] * B + gl * SPL;
#pragma unroll
          for (int k = 0; k < SPL; ++k) sl[u][k] = p[k];
        }
      }
#pragma unroll
      for (int u = 0; u < QL; ++u) {
        if (!want[u]) continue;  // uniform within the query's lane group
        ++probes[u];
        int mk = -1;
#pragma unroll
        for (int k = SPL - 1; k >= 0; --k)
          if (sl[u][k].x == x[u]) mk = k;
        const uint64_t m = (__ballot(mk >= 0) >> gshift) & gmask;
        if (m) {
          winner[u] = __ffsll((unsigned long long)m) - 1;
          if (gl == winner[u]) {
            uint64_t v = 0;
#pragma unroll
            for (int k = 0; k < SPL; ++k)
              if (k == mk) v = sl[u][k].y;
            val[u] = v;
          }
          hit[u] = true;
        }
      }
    }
    // Then the stash, one more probe for a query its bins did not answer.  A
    // stash has at most 64 entries: each lane of the wavefront holds one key,
    // and each unanswered query is compared with all of them in one ballot.
    // A wavefront whose unanswered queries are of several tables (a group)
    // searches per query group instead.
    if (EXT && g.stash_n) {
#pragma unroll
      for (int u = 0; u < QL; ++u) {  // every lane of the wavefront takes each pass
        const bool need = x[u] != kEmpty && !hit[u];
        if (need) ++probes[u];
        const uint64_t needm = __ballot(need && gl == 0);
        if (needm) {
          const uint32_t t = need ? table_of(op_table, qv[u]) : 0u;
          const uint32_t t0 = __shfl(t, __ffsll((unsigned long long)needm) - 1, 64);
          if (__ballot(need && t != t0) == 0) {
            if (g.stash_cnt[t0]) {
              const uint32_t sb = t0 * g.stash_n;
              const uint64_t ek = lane < (int)g.stash_n ? g.stash[sb + lane].x : kEmpty;
              uint64_t rem = needm, got = 0, gv = 0;
              while (rem) {  // wavefront-uniform
                const int l = __ffsll((unsigned long long)rem) - 1;
                const uint64_t mm = __ballot(ek == __shfl(x[u], l, 64));
                if (mm) {
                  if (lane == l) gv = g.stash[sb + __ffsll((unsigned long long)mm) - 1].y;
                  got |= 1ull << l;
                }
                rem &= rem - 1;
              }
              if ((got >> gshift) & 1ull) {  // found by this query's group leader
                hit[u] = true;
                winner[u] = 0;
                if (gl == 0) val[u] = gv;
              }
            }
          } else if (need) {
            const uint32_t e = stash_find(g, t, x[u], gl, LPP, [&](bool p) {
              return (uint64_t)((__ballot(p) >> gshift) & gmask);
            });
            if (e != kNone) {
              hit[u] = true;
              winner[u] = 0;
              val[u] = g.stash[e].y;
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < QL; ++u) {
      if (active[u] && gl == winner[u]) {
        if (B == 1) ((uint32_t*)out)[qv[u]] = (uint32_t)val[u];
        else ((uint64_t*)out)[qv[u]] = val[u];
        found[qv[u]] = hit[u] ? 1 : 0;
      }
      if (active[u] && gl == 0) {
        probes_acc += probes[u];
        hits_acc += hit[u] ? 1 : 0;
      }
    }
  }
  DevStatLine& sl = st->s[blockIdx.x % kStatStripes];
  block_add2(probes_acc, hits_acc, &sl.v[S_LOOKUP_PROBES], &sl.v[S_LOOKUP_HITS]);
}

template <int B, int LPP, int H>
static void lookup_go(const Geo& g, const uint64_t* keys, uint64_t n, void* out, uint8_t* found,
                      DevStats* st, const uint32_t* op_table, const uint2* tdesc, hipStream_t s) {
  const uint64_t blocks = (n * LPP + 256 * lookup_queries_per_group<B, LPP>() - 1) /
                          (256 * lookup_queries_per_group<B, LPP>());
  const uint32_t grid = (uint32_t)std::min<uint64_t>(blocks, 8192);
  if (g.stash_n || g.hash_bias)
    hipLaunchKernelGGL((k_lookup<B, LPP, H, true>), dim3(grid), dim3(256), 0, s, g, keys, n, out,
                       found, st, op_table, tdesc);
  else
    hipLaunchKernelGGL((k_lookup<B, LPP, H, false>), dim3(grid), dim3(256), 0, s, g, keys, n, out,
                       found, st, op_table, tdesc);
}

hipError_t launch_lookup(const Geo& g, const uint64_t* keys, uint64_t n, void* out,
                         uint8_t* found, uint32_t lpp, DevStats* st, const uint32_t* op_table,
                         const uint2* tdesc, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const bool wide = (lpp == g.B);
  switch (g.B) {
    case 1:
      if (g.H == 2) lookup_go<1, 1, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      else if (g.H == 3) lookup_go<1, 1, 3>(g, keys, n, out, found, st, op_table, tdesc, s);
      else lookup_go<1, 1, 4>(g, keys, n, out, found, st, op_table, tdesc, s);
      break;
    case 2:
      if (wide) lookup_go<2, 2, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      else lookup_go<2, 1, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      break;
    case 4:
      if (wide) lookup_go<4, 4, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      else lookup_go<4, 1, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      break;
    case 8:
      if (wide) lookup_go<8, 8, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      else lookup_go<8, 1, 2>(g, keys, n, out, found, st, op_table, tdesc, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// round bookkeeping
// ---------------------------------------------------------------------------
// Round start, done by block 0 of the round's first kernel (the fresh or
// delete planner): the next list's segment counts are zeroed (the commit
// kernel of this round is the first to touch them), and an arena overflow of
// the previous round is remembered for the host and cleared.  The first round
// of a sub-batch resets the sub-batch's counters instead; its pending list is
// every op in order, so position and op index coincide.
__device__ __forceinline__ void round_start(const Round& r) {
  if (threadIdx.x < kStripes) r.next_cnt[threadIdx.x * kStripeWords] = 0;
  if (threadIdx.x != 0) return;
  Ctr* c = r.ctr;
  if (r.first) {  // a new sub-batch
    c->rounds = 0;
    c->overflow_seen = 0;
  } else if (c->overflow) {
    c->overflow_seen = 1;
  }
  c->overflow = 0;
}
__device__ __forceinline__ void zero_op_counters(const Round& r, uint32_t i) {
  r.op_views[i] = 0;
  r.op_lost[i] = 0;
  r.op_kicks[i] = 0;
  r.op_retries[i] = 0;
  r.op_twins[i] = 0;
}


// ---------------------------------------------------------------------------
// plan emission helpers (called by one lane)
// ---------------------------------------------------------------------------
// Every eviction-planner workgroup owns a fixed region of the plan arena
// (cap / gridDim.x entries) and fills it in order: no device-wide counter.  A
// plan that does not fit marks the round void; the host then grows the arena
// and the round is planned again.  win[0] = next free entry, win[1] = region
// end.
__device__ __forceinline__ void region_init(uint32_t* win, uint32_t cap) {
  const uint32_t per = cap / gridDim.x;
  win[0] = blockIdx.x * per;
  win[1] = win[0] + per;
}

__device__ __forceinline__ void claim(const Geo& g, const Round& r, uint32_t bin, uint32_t i) {
  atomicMin(&g.owner[bin], r.tag | (unsigned long long)i);
}

// A failed insert's key goes to the first free entry of its table's stash
// (in the round's snapshot), if there is one; the entry is claimed like a bin.
// Returns the entry's index in the stash array, or kNone.  One lane.
__device__ uint32_t stash_take(const Geo& g, const Round& r, uint32_t i) {
  if (g.stash_n == 0) return kNone;
  const uint32_t t = table_of(r.op_table, i);
  if (g.stash_cnt[t] >= g.stash_n) return kNone;
  const uint32_t sb = t * g.stash_n;
  for (uint32_t j = 0; j < g.stash_n; ++j)
    if (g.stash[sb + j].x == kEmpty) {
      atomicMin(&g.stash_owner[sb + j], r.tag | (unsigned long long)i);
      return sb + j;
    }
  return kNone;
}

// ---------------------------------------------------------------------------
// k_plan_fresh: B lanes per op, placement without eviction
// ---------------------------------------------------------------------------
template <int B>
struct GroupCtx {
  int lane, sl, gshift;
  __device__ __forceinline__ uint32_t ballot(bool p) const {
    return (uint32_t)((__ballot(p) >> gshift) & ((B == 64) ? ~0ull : ((1ull << B) - 1)));
  }
};

// The keys of one bin as the L lanes of an op's group hold them: lane j has
// slots j, j + L, j + 2L, ... (S = B / L of them), so each of the S loads of
// the group reads one contiguous stretch of the bin's line.
template <int B, int L>
struct BinKeys {
  static constexpr int S = B / L;
  uint64_t k[S];
  __device__ __forceinline__ void load(const Geo& g, uint32_t bin, int sl) {
    const ulonglong2* p = g.slots + (uint64_t)bin * B + sl;
#pragma unroll
    for (int q = 0; q < S; ++q) k[q] = p[q * L].x;
  }
  // slots whose key is v, as a B-bit mask (bit = slot index)
  __device__ __forceinline__ uint32_t match(const GroupCtx<L>& G, uint64_t v) const {
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < S; ++q) m |= G.ballot(k[q] == v) << (q * L);
    return m;
  }
  // the key in slot `slot` (group-uniform)
  __device__ __forceinline__ uint64_t at(const GroupCtx<L>& G, uint32_t slot) const {
    uint64_t v = k[0];
#pragma unroll
    for (int q = 1; q < S; ++q)
      if (slot / L == (uint32_t)q) v = k[q];
    return __shfl(v, G.gshift + (int)(slot % L), 64);
  }
};

// EXT: the instance for upserts, stashes and biased hashes; the plain one
// carries none of their code (the host picks by the table and the call).
template <int B, int H, bool EXT>
__global__ __launch_bounds__(256) void k_plan_fresh(Geo g, Round r) {
  constexpr int L = fresh_lanes(B);
  using Keys = BinKeys<B, L>;
  GroupCtx<L> G;
  G.lane = threadIdx.x & 63;
  G.sl = G.lane % L;
  G.gshift = G.lane - G.sl;
  if (blockIdx.x == 0) round_start(r);
  Pending P;
  P.init(r);
  constexpr uint32_t opb = 256 / L, opw = 64 / L;
  const uint32_t passes = (P.n + opb - 1) / opb;
  // pass c takes positions [c opb, (c + 1) opb); rounds after the first run a
  // capped grid, so a workgroup may take several passes
  for (uint32_t c = blockIdx.x; c < passes; c += gridDim.x) {
    const uint32_t pi = P.at(c * opb + threadIdx.x / L);
    const bool active = pi != kNone;
    const uint32_t i = active ? pi : 0u;
    if (r.first && active && (threadIdx.x % L) == 0) zero_op_counters(r, i);
    const uint64_t x = active ? r.keys[i] : kEmpty;
    const bool leader = G.sl == 0;
    const bool bad = x == kEmpty;  // reserved key: rejected, no plan
    const uint32_t hc_flag = (g.scheme == CK_QUEUE) ? MV_HC : 0;
    // up to two moves (slot | flags << 8), group-uniform, kept in registers;
    // the written record is always this op's own key and value
    uint32_t b0 = 0, f0 = 0, b1 = 0, f1 = 0;
    uint32_t nm = 0, views = 0, twins = 0;
    bool placed = false;
    const Tab T = active ? tab_of(g, r.op_table, r.tdesc, i) : Tab{0u, g.n};
    // upsert: the key's bins are searched in hash order first.  A stored key
    // gets its new value in place (both copies of a ghost pair); an absent
    // one is inserted as below, having viewed all H bins, and its plan also
    // claims the key's first bin (kHdrKeyClaim), so that of two upserts of
    // one new key in a round the later one loses and then finds the key.
    const bool ups = EXT && r.upsert && active && !bad;
    bool updated = false;
    uint32_t key_bin = 0, stash_e = kNone;
    if (ups) {
      uint32_t h[H];
      hash_key<H, EXT>(g, T, x, h);
      key_bin = h[0];
#pragma unroll
      for (int hi = 0; hi < H; ++hi) {
        Keys sv;
        sv.load(g, h[hi], G.sl);
        const uint32_t m = sv.match(G, x);
        if (m) {
          const uint32_t slot = ffs32(m);
          b0 = h[hi]; f0 = slot | (MV_VALUE << 8); nm = 1;
          if (g.ghost && ((g.meta[h[hi]] >> slot) & 1u)) {
            const uint32_t tb = h[hi ^ 1];
            Keys ts;
            ts.load(g, tb, G.sl);
            b1 = tb; f1 = ffs32(ts.match(G, x)) | (MV_VALUE << 8); nm = 2;
          }
          views = (uint32_t)hi + 1;
          updated = true;
          break;
        }
      }
      if (!updated && g.stash_n) {  // then the stash, one more view
        stash_e = stash_find(g, table_of(r.op_table, i), x, G.sl, L,
                             [&](bool p) { return (uint64_t)G.ballot(p); });
        if (stash_e != kNone) {
          views = (uint32_t)H + 1;
          updated = true;
        }
      }
    }
    // rattle-kicking has no separate fresh phase: every op goes to the walk
    if (active && !bad && !updated && g.scheme != CK_RATTLE) {
      uint32_t h[H];
      hash_key<H, EXT>(g, T, x, h);
      if (g.ghost) {
        Keys s0, s1;
        s0.load(g, h[0], G.sl);
        s1.load(g, h[1], G.sl);
        views = 2;
        const uint32_t e0 = s0.match(G, kEmpty), e1 = s1.match(G, kEmpty);
        if (e0 && e1) {
          b0 = h[0]; f0 = ffs32(e0) | ((MV_DUP | hc_flag) << 8);
          b1 = h[1]; f1 = ffs32(e1) | ((MV_DUP | hc_flag) << 8);
          nm = 2;
          placed = true;
        } else if (e0) {
          b0 = h[0]; f0 = ffs32(e0) | (hc_flag << 8); nm = 1;
          placed = true;
        } else if (e1) {
          b0 = h[1]; f0 = ffs32(e1) | (hc_flag << 8); nm = 1;
          placed = true;
        } else {
          const uint32_t full = (1u << B) - 1;
          const uint32_t d0 = g.meta[h[0]] & full, d1 = g.meta[h[1]] & full;
          if (d0 || d1) {
            const int w = d0 ? 0 : 1;
            const uint32_t b = w == 0 ? h[0] : h[1];
            const uint32_t ds = ffs32(d0 ? d0 : d1);
            const uint64_t dk = w == 0 ? s0.at(G, ds) : s1.at(G, ds);
            uint32_t hd[2];
            hash_key<2, EXT>(g, T, dk, hd);
            const uint32_t tb = hd[0] == b ? hd[1] : hd[0];
            Keys ts;
            ts.load(g, tb, G.sl);
            const uint32_t tm = ts.match(G, dk);
            b0 = tb; f0 = ffs32(tm) | (MV_DUPCLR << 8);
            b1 = b; f1 = ds | (hc_flag << 8);
            nm = 2;
            twins = 1;
            placed = true;
          }
        }
      } else if (g.balance || g.scheme == CK_QUEUE) {
        Keys s0, s1;
        s0.load(g, h[0], G.sl);
        s1.load(g, h[1], G.sl);
        views = 2;
        const uint32_t e0 = s0.match(G, kEmpty), e1 = s1.match(G, kEmpty);
        const int o0 = B - __popc(e0), o1 = B - __popc(e1);
        if (o0 < B || o1 < B) {
          if (o0 <= o1) { b0 = h[0]; f0 = ffs32(e0) | (hc_flag << 8); }
          else { b0 = h[1]; f0 = ffs32(e1) | (hc_flag << 8); }
          nm = 1;
          placed = true;
        }
      } else {
#pragma unroll
        for (int hi = 0; hi < H; ++hi) {
          Keys sv;
          sv.load(g, h[hi], G.sl);
          ++views;
          const uint32_t e = sv.match(G, kEmpty);
          if (e) {
            b0 = h[hi]; f0 = ffs32(e) | (hc_flag << 8); nm = 1;
            placed = true;
            break;
          }
        }
      }
    }
    // ops that need a kick-out go to this wavefront's region of the evict
    // list, in op order, with its count beside it (no shared counter)
    {
      const int lane = threadIdx.x & 63;
      const uint32_t u = c * 4 + (threadIdx.x >> 6);
      const bool ev = active && leader && !bad && !placed && !updated;
      const uint64_t bal = __ballot(ev);
      if (ev) r.evict[(size_t)u * opw + __popcll(bal & ((1ull << lane) - 1))] = i;
      if (lane == 0) r.evict_cnt[u] = (uint32_t)__popcll(bal);
    }
    if (active && leader) {
      const bool key_claim = ups && !updated;
      const bool in_stash = stash_e != kNone;
      const uint32_t st = bad ? PL_FAIL : (updated ? PL_UPDATED : (placed ? PL_OK : PL_EVICT));
      r.hdr[i] = make_uint4(
          hdr_pack(st, twins, nm) | (key_claim ? kHdrKeyClaim : 0u) | (in_stash ? kHdrStash : 0u),
          views + (key_claim ? (uint32_t)H + (g.stash_n ? 1u : 0u) : 0u), b0,
          in_stash ? stash_e : f0);
      if (in_stash) atomicMin(&g.stash_owner[stash_e], r.tag | (unsigned long long)i);
      if (placed || updated) {
        if (nm > 0) claim(g, r, b0, i);
        if (nm > 1) {
          r.imv[(size_t)i * kExtraInline] = IMove{b1, f1};
          claim(g, r, b1, i);
        }
      }
      if (key_claim) claim(g, r, key_bin, i);
    }
  }
}

// ---------------------------------------------------------------------------
// The ops of one round that need an eviction plan: fresh-planner wavefront b
// put its evict_cnt[b] ops at evict[b * opw + j], j < evict_cnt[b] (opw = 64 /
// fresh_lanes(B) ops per wavefront).  Positions are numbered slot-major, q = j * nb + b (nb
// wavefronts), so each stretch of q holds one slot index of every wavefront.  Eviction-planner
// workgroup w takes q = w, w + gridDim.x, w + 2 gridDim.x, ...: an even
// sample of every slot layer, hence an equal share of the occupied
// positions; its item k is its k-th occupied position.  The wavefront checks
// 64 positions per step (one per lane) and ballots the occupied ones.
// ---------------------------------------------------------------------------
struct EvictWork {
  const uint32_t* list = nullptr;
  const uint32_t* cnt = nullptr;
  uint64_t npos = 0;   // fresh-planner wavefronts * opw
  uint32_t opb = 1, nb = 1;
  uint32_t c0 = 0;     // window: positions w + (64 c0 + lane) gridDim.x
  uint64_t vmask = 0;  // occupied positions of the window
  uint32_t base = 0;   // items before the window
  uint32_t wtot = 0;   // items in the window

  __device__ void window(uint32_t c) {
    c0 = c;
    const int lane = threadIdx.x & 63;
    const uint64_t q = (uint64_t)blockIdx.x + ((uint64_t)c0 * 64 + lane) * gridDim.x;
    bool v = false;
    if (q < npos) v = (uint32_t)(q / nb) < cnt[q % nb];
    vmask = (uint64_t)__ballot(v);
    wtot = (uint32_t)__popcll(vmask);
  }
  __device__ void init(const Round& r, uint32_t opw) {  // all 64 lanes together
    Pending P;
    P.init(r);
    list = r.evict;
    cnt = r.evict_cnt;
    opb = opw;
    nb = (P.n + opb - 1) / opb;
    npos = (uint64_t)nb * opb;
    base = 0;
    window(0);
  }
  // op index of item k, or kNone past the end; k must not decrease
  __device__ uint32_t item(uint32_t k) {
    while (k >= base + wtot) {
      if ((uint64_t)blockIdx.x + (uint64_t)(c0 + 1) * 64 * gridDim.x >= npos) return kNone;
      base += wtot;
      window(c0 + 1);
    }
    const int lane = threadIdx.x & 63;
    const uint32_t rel = k - base;
    const uint32_t below = (uint32_t)__popcll(vmask & ((1ull << lane) - 1));
    const bool hit = ((vmask >> lane) & 1ull) && below == rel;
    const uint32_t t = (uint32_t)(__ffsll((unsigned long long)__ballot(hit)) - 1);
    const uint64_t q = (uint64_t)blockIdx.x + ((uint64_t)c0 * 64 + t) * gridDim.x;
    return list[(q % nb) * opb + q / nb];
  }
};

// ---------------------------------------------------------------------------
// Walk planners (random kicking, queue-kicking, rattle-kicking): a
// wavefront runs 64 / kWalkW walks side by side, kWalkW lanes each (a group);
// lanes < B of a group hold the slots of the bin the walk is viewing.  A
// walk logs its moves; a later view of a bin it already wrote shows its own
// writes (the overlay).  The first kWalkLdsLog moves of a walk are logged in
// LDS, longer chains continue in workgroup scratch.
// ---------------------------------------------------------------------------
constexpr int kWalkW = 8;
constexpr uint32_t kWalkLdsLog = 32;

// Orders LDS and memory accesses of the lanes of one wavefront (the planner
// workgroups are single wavefronts, so this is a full workgroup barrier);
// valid in divergent code.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Arena regions shared by the workgroup's planners.
__device__ __forceinline__ uint32_t region_take(uint32_t* win, uint32_t n, Ctr* ctr) {
  if (n == 0) return 0;
  const uint32_t off = atomicAdd(&win[0], n);
  if (off + n > win[1]) {
    atomicOr(&ctr->overflow, 1u);
    return kNone;
  }
  return off;
}

// A walk's move log: entries < kWalkLdsLog in LDS, the rest in scratch, and
// a filter of the bins it wrote (one bit per bin hash; a view of a bin whose
// bit is clear has nothing to overlay).  2048 bits, or 8192 for random
// kicking in single-slot bins, whose walks run to a thousand kicks: there a
// filter half full sent every other view through a scan of the whole log.
constexpr uint32_t kWalkMapWords = 64;       // 2048 bits
constexpr uint32_t kWalkMapWordsLong = 256;  // 8192 bits
// Those long walks also keep a second filter of 65536 bits (another hash of
// the bin) in their scratch, read only when the first one's bit is set: a
// whole-log scan then happens about once in 500 views instead of once in 8.
constexpr uint32_t kWalkMap2Words = 2048;
__host__ __device__ __forceinline__ uint32_t walk_map_words(const Geo& g) {
  return (g.scheme == CK_RANDOM_WALK && g.B == 1) ? kWalkMapWordsLong : kWalkMapWords;
}
struct WalkLog {
  uint64_t* key;    // LDS, kWalkLdsLog each
  uint64_t* aux;
  uint32_t* bin;
  uint32_t* sf;     // slot | flags << 8
  int* last;        // LDS [8]
  uint32_t* misc;   // LDS [8]: 0 hc adds
  uint32_t* wmap;   // LDS [walk_map_words]
  uint32_t mshift;  // 32 - log2(filter bits)
  uint32_t* gmap2;  // scratch [kWalkMap2Words], the second filter, or null
  uint64_t* gkey;   // scratch, indexed from 0 (entries < kWalkLdsLog unused)
  uint64_t* gaux;
  uint32_t* gbin;
  uint32_t* gsf;
  __device__ __forceinline__ uint64_t& k(uint32_t j) const { return j < kWalkLdsLog ? key[j] : gkey[j]; }
  __device__ __forceinline__ uint64_t& a(uint32_t j) const { return j < kWalkLdsLog ? aux[j] : gaux[j]; }
  __device__ __forceinline__ uint32_t& b(uint32_t j) const { return j < kWalkLdsLog ? bin[j] : gbin[j]; }
  __device__ __forceinline__ uint32_t& f(uint32_t j) const { return j < kWalkLdsLog ? sf[j] : gsf[j]; }
  __device__ __forceinline__ uint32_t mbit(uint32_t b) const { return (b * 0x9E3779B1u) >> mshift; }
  __device__ static __forceinline__ uint32_t mbit2(uint32_t b) { return (b * 0x85EBCA6Bu) >> 16; }
  __device__ __forceinline__ bool maybe_written(uint32_t b) const {
    const uint32_t h = mbit(b);
    if (!((wmap[h >> 5] >> (h & 31)) & 1u)) return false;
    if (!gmap2) return true;
    const uint32_t h2 = mbit2(b);
    return (gmap2[h2 >> 5] >> (h2 & 31)) & 1u;
  }
  __device__ __forceinline__ void mark(uint32_t b) const {  // one lane
    const uint32_t h = mbit(b);
    wmap[h >> 5] |= 1u << (h & 31);
    if (gmap2) {
      const uint32_t h2 = mbit2(b);
      atomicOr(&gmap2[h2 >> 5], 1u << (h2 & 31));
    }
  }
};

template <int B, int H, bool EXT>
struct WalkPlanner {
  static constexpr int W = kWalkW;
  const Geo& g;
  const Round& r;
  WalkLog L;
  int gl, gb;          // lane within the group, the group's first lane
  uint32_t cap;        // log capacity
  uint32_t nm = 0;     // moves logged
  uint32_t views = 0, kicks = 0, twins = 0, draws = 0;
  uint64_t op = 0;     // global insert index
  Tab T{0u, 0u};       // the op's table
  bool overflow = false;

  // bin view state (group lanes < B)
  uint64_t vkey = kEmpty, vaux = 0;
  bool vdup = false;
  int vprev = -1;      // log index of the last write to this lane's slot
  uint32_t vhc = 0;    // hit counter of the viewed bin (group-uniform)
  uint32_t vmeta = 0;  // metadata word of the viewed bin, as read (group-uniform)
  uint32_t vbin = kNone;

  __device__ WalkPlanner(const Geo& g_, const Round& r_, WalkLog l, uint32_t cap_)
      : g(g_), r(r_), L(l), gl(threadIdx.x % W), gb(threadIdx.x - threadIdx.x % W), cap(cap_) {}

  __device__ __forceinline__ uint32_t ballotB(bool p) const {
    return (uint32_t)((__ballot(gl < B && p) >> gb) & ((1ull << B) - 1));
  }
  template <class V>
  __device__ __forceinline__ V gshfl(V v, uint32_t src) const {
    return __shfl(v, gb + (int)src, 64);
  }

  // Load bin b into group lanes < B, applying this plan's earlier writes.
  // `count` = true makes it a bin view (Sec. 3 cost unit).
  __device__ void load(uint32_t b, bool count) {
    if (count) ++views;
    ulonglong2 s = make_ulonglong2(kEmpty, 0ull);
    if (gl < B) s = g.slots[(uint64_t)b * B + gl];
    uint32_t m = (g.ghost || g.scheme == CK_QUEUE) ? g.meta[b] : 0u;
    bool dup = gl < B && ((m >> gl) & 1u);
    int prev = -1;
    uint32_t hcadd = 0;
    if (nm > 0 && L.maybe_written(b)) {
      if (gl < 8) L.last[gl] = -1;
      if (gl == 0) L.misc[0] = 0;
      wave_sync();
      for (uint32_t j = gl; j < nm; j += W) {
        if (L.b(j) == b) {
          const uint32_t sf = L.f(j);
          const uint32_t f = sf >> 8;
          if (!(f & MV_DUPCLR)) atomicMax(&L.last[sf & 0xFF], (int)j);
          if (f & MV_HC) atomicAdd(&L.misc[0], 1u);
        }
      }
      wave_sync();
      if (gl < B) {
        prev = L.last[gl];
        if (prev >= 0) {
          s.x = L.k(prev);
          s.y = L.a(prev);
          dup = (L.f(prev) >> 8) & MV_DUP;
        }
      }
      hcadd = L.misc[0];
      wave_sync();
    }
    vkey = s.x;
    vaux = s.y;
    vmeta = m;
    vdup = dup && s.x != kEmpty;
    vprev = prev;
    vhc = ((m >> 24) + hcadd) & 0xFFu;
    vbin = b;
  }

  __device__ __forceinline__ uint32_t empty_mask() const { return ballotB(vkey == kEmpty); }
  __device__ __forceinline__ uint32_t dup_mask() const { return ballotB(vdup); }
  __device__ __forceinline__ bool terminal() const {
    return empty_mask() != 0 || (g.ghost && dup_mask() != 0);
  }
  __device__ __forceinline__ uint64_t slot_key(uint32_t s) const { return gshfl(vkey, s); }
  __device__ __forceinline__ uint64_t slot_aux(uint32_t s) const { return gshfl(vaux, s); }

  // Log a write of (key, aux) to slot s of the currently viewed bin.
  __device__ void emit_here(uint32_t s, uint64_t k, uint64_t a, uint32_t flags) {
    const int prev = gshfl(vprev, s);
    if (nm >= cap) { overflow = true; return; }
    if (gl == 0) {
      if (prev >= 0) L.f(prev) |= ((uint32_t)MV_SUPERSEDED << 8);
      L.k(nm) = k;
      L.a(nm) = a;
      L.b(nm) = vbin;
      L.f(nm) = s | (flags << 8);
      L.mark(vbin);
    }
    ++nm;
    // keep the view coherent with the write (the walk may read this bin again)
    if (gl == (int)s) {
      vkey = k;
      vaux = a;
      vdup = (flags & MV_DUP) != 0;
      vprev = (int)nm - 1;
    }
    if (flags & MV_HC) vhc = (vhc + 1) & 0xFFu;
    wave_sync();
  }
  __device__ void emit_other(uint32_t b, uint32_t s, uint64_t k, uint64_t a, uint32_t flags) {
    if (nm >= cap) { overflow = true; return; }
    if (gl == 0) {
      L.k(nm) = k;
      L.a(nm) = a;
      L.b(nm) = b;
      L.f(nm) = s | (flags << 8);
      L.mark(b);
    }
    ++nm;
    wave_sync();
  }

  // Drop the duplicate in slot s of the viewed bin and put (k, a) there; the
  // twin copy in the duplicate key's other bin loses its mark (Sec. 4).
  __device__ void replace_dup(uint32_t s, uint64_t k, uint64_t a, uint32_t flags) {
    const uint64_t dk = slot_key(s);
    uint32_t hd[2];
    hash_key<2, EXT>(g, T, dk, hd);
    const uint32_t here = vbin;
    const uint32_t tb = hd[0] == here ? hd[1] : hd[0];
    ulonglong2 ts = make_ulonglong2(kEmpty, 0ull);
    if (gl < B) ts = g.slots[(uint64_t)tb * B + gl];
    const uint32_t tm = ballotB(ts.x == dk);
    emit_other(tb, ffs32(tm), 0, 0, MV_DUPCLR);
    ++twins;
    emit_here(s, k, a, flags);
  }

  // Put (k, a) into the viewed terminal bin: a free slot first, else a duplicate.
  __device__ void place_terminal(uint64_t k, uint64_t a, uint32_t flags) {
    const uint32_t e = empty_mask();
    if (e) emit_here(ffs32(e), k, a, flags);
    else replace_dup(ffs32(dup_mask()), k, a, flags);
  }

  // Ops reach the eviction planners only after k_plan_fresh found no room
  // for them in the same snapshot, so their fresh views need no re-reading:
  // first fit viewed all H bins, ghost and load-balanced inserts both bins.
  __device__ __forceinline__ uint32_t fresh_views_full() const {
    return (g.ghost || g.balance || g.scheme == CK_QUEUE) ? 2u : (uint32_t)H;
  }

  // ---- random kicking (Sec. 1; d-ary: victim moves to one of its other bins)
  __device__ uint32_t random_walk(uint64_t x, uint64_t xa, const uint32_t* h) {
    views = fresh_views_full();
    uint32_t cur = h[uniform_choice(g, op, draws, H)];
    load(cur, false);
    uint64_t ck = x, ca = xa;
    for (;;) {
      if (kicks == g.max_chain) return PL_FAIL;
      const uint32_t s = uniform_choice(g, op, draws, B);
      const uint64_t vk = slot_key(s), va = slot_aux(s);
      emit_here(s, ck, ca, 0);
      if (overflow) return PL_FAIL;
      ++kicks;
      ck = vk;
      ca = va;
      uint32_t hv[H];
      hash_key<H, EXT>(g, T, ck, hv);
      uint32_t oth[H];
      uint32_t no = 0;
      for (int q = 0; q < H; ++q)
        if (hv[q] != cur) oth[no++] = hv[q];
      cur = oth[uniform_choice(g, op, draws, no)];
      load(cur, true);
      if (terminal()) {
        place_terminal(ck, ca, 0);
        return overflow ? PL_FAIL : PL_OK;
      }
    }
  }

  // ---- queue-kicking with hit counters and hit balancing (Sec. 6)
  __device__ uint32_t queue_kick(uint64_t x, uint64_t xa, const uint32_t* h) {
    views = fresh_views_full();
    const uint32_t hc0 = g.meta[h[0]] >> 24, hc1 = g.meta[h[1]] >> 24;
    uint32_t t = hc0 <= hc1 ? h[0] : h[1];
    load(t, false);
    uint64_t ck = x, ca = xa;
    for (;;) {
      if (kicks == g.max_chain) return PL_FAIL;
      const uint32_t s = vhc % B;
      const uint64_t vk = slot_key(s), va = slot_aux(s);
      emit_here(s, ck, ca, MV_HC);
      if (overflow) return PL_FAIL;
      ++kicks;
      ck = vk;
      ca = va;
      uint32_t hv[2];
      hash_key<2, EXT>(g, T, ck, hv);
      t = hv[0] == t ? hv[1] : hv[0];
      load(t, true);
      if (terminal()) {
        place_terminal(ck, ca, MV_HC);
        return overflow ? PL_FAIL : PL_OK;
      }
    }
  }

  // ---- rattle-kicking (Sec. 7), single-slot bins
  __device__ uint32_t rattle(uint64_t x, uint64_t xa) {
    uint64_t ck = x, ca = with_rattle(xa, 0);
    uint32_t tries = 0;
    for (;;) {
      if (tries == g.max_chain) return PL_FAIL;
      uint32_t hv[H];
      hash_key<H, EXT>(g, T, ck, hv);
      uint32_t rr = rattle_of(ca);
      const uint32_t b = hv[rr % H];
      rr = (rr + 1) & 0xFFFF;
      ca = with_rattle(ca, rr);
      ++tries;
      load(b, true);
      const uint64_t yk = slot_key(0), ya = slot_aux(0);
      if (yk == kEmpty) {
        emit_here(0, ck, ca, 0);
        return overflow ? PL_FAIL : PL_OK;
      }
      if (rr > rattle_of(ya)) {
        emit_here(0, ck, ca, 0);
        if (overflow) return PL_FAIL;
        ++kicks;
        ck = yk;
        ca = ya;
      }
    }
  }

  // Copy the logged moves to the arena, write the header and claim bins.
  __device__ void finish(uint32_t i, uint32_t status, uint32_t* win,
                         unsigned long long* wg_views) {
    if (status != PL_OK) nm = 0;
    uint32_t o = 0;
    if (gl == 0) o = region_take(win, nm, r.ctr);
    const uint32_t off = gshfl(o, 0);
    if (off != kNone) {
      for (uint32_t j = gl; j < nm; j += W) {
        Move mv;
        mv.key = L.k(j);
        mv.aux = L.a(j);
        mv.bin = L.b(j);
        mv.slot = (uint8_t)(L.f(j) & 0xFF);
        mv.flags = (uint8_t)(L.f(j) >> 8);
        mv.pad = 0;
        r.arena[off + j] = mv;
        claim(g, r, mv.bin, i);
      }
    }
    if (gl == 0) {
      // a failed chain's key goes to the stash if it has room
      const uint32_t se = (EXT && status == PL_FAIL) ? stash_take(g, r, i) : kNone;
      // an upsert's plan adds the presence check's views and its key claim
      // (made by the fresh planner)
      r.hdr[i] = make_uint4(
          hdr_pack(se != kNone ? PL_STASHED : status, status == PL_OK ? twins : 0, nm) |
              kHdrArena | ((EXT && r.upsert) ? kHdrKeyClaim : 0u) | (se != kNone ? kHdrStash : 0u),
          views + ((EXT && r.upsert) ? (uint32_t)H + (g.stash_n ? 1u : 0u) : 0u), off,
          status == PL_OK ? kicks : (se != kNone ? se : 0u));
      r.hdr_spawn[i] = make_uint2(0u, 0u);
      atomicAdd(wg_views, (unsigned long long)views);
    }
    wave_sync();
  }
};

__host__ __device__ inline size_t walk_group_lds_bytes(const Geo& g) {
  return kWalkLdsLog * 24 + 16 * 4 + walk_map_words(g) * 4;
}
static size_t walk_group_scratch_bytes(const Geo& g) {
  const size_t map2 = walk_map_words(g) == kWalkMapWordsLong ? kWalkMap2Words * 4 : 0;
  return ((size_t)(g.max_chain + 8) * 24 + map2 + 255) & ~(size_t)255;
}

template <int B, int H, bool EXT>
__global__ __launch_bounds__(64) void k_plan_walk(Geo g, Round r) {
  constexpr int W = kWalkW;
  constexpr int P = 64 / W;
  extern __shared__ uint64_t lds64[];
  __shared__ uint32_t win[2];
  __shared__ unsigned long long s_views;  // bins viewed by this workgroup's plans
  const int lane = threadIdx.x;
  const int gi = lane / W;
  const uint32_t cap = g.max_chain + 8;
  const uint32_t mwords = walk_map_words(g);
  WalkLog L;
  {
    char* base = (char*)lds64 + (size_t)gi * walk_group_lds_bytes(g);
    L.key = (uint64_t*)base;
    L.aux = L.key + kWalkLdsLog;
    L.bin = (uint32_t*)(L.aux + kWalkLdsLog);
    L.sf = L.bin + kWalkLdsLog;
    L.last = (int*)(L.sf + kWalkLdsLog);
    L.misc = (uint32_t*)(L.last + 8);
    L.wmap = L.misc + 8;
    L.mshift = mwords == kWalkMapWordsLong ? 19u : 21u;
    char* sc = (char*)r.wg_scratch + (size_t)blockIdx.x * r.wg_scratch_bytes +
               (size_t)gi * (r.wg_scratch_bytes / P);
    L.gkey = (uint64_t*)sc;
    L.gaux = L.gkey + cap;
    L.gbin = (uint32_t*)(L.gaux + cap);
    L.gsf = L.gbin + cap;
    L.gmap2 = mwords == kWalkMapWordsLong ? L.gsf + cap : nullptr;
  }
  if (lane == 0) {
    region_init(win, r.arena_cap);
    s_views = 0;
  }
  wave_sync();
  EvictWork Wk;
  Wk.init(r, 64 / fresh_lanes(B));
  // the group's op of batch kb is item kb + gi; item() is wave-uniform
  auto batch_item = [&](uint32_t kb) -> uint32_t {
    uint32_t mine = kNone;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint32_t v = Wk.item(kb + (uint32_t)p);
      if (gi == p) mine = v;
    }
    return mine;
  };
  // software-pipelined: the next batch's ops and keys are fetched while the
  // current walks run
  uint32_t i_nx = batch_item(0);
  uint64_t x_nx = i_nx != kNone ? r.keys[i_nx] : 0ull;
  for (uint32_t kb = 0;; kb += P) {
    if (__ballot(i_nx != kNone) == 0) break;  // wave-uniform
    const uint32_t i = i_nx;
    const uint64_t x = x_nx;
    i_nx = batch_item(kb + P);
    if (i_nx != kNone) x_nx = r.keys[i_nx];
    for (uint32_t j = lane % W; j < mwords; j += W) L.wmap[j] = 0;
    if (L.gmap2)
      for (uint32_t j = lane % W; j < kWalkMap2Words; j += W) L.gmap2[j] = 0;
    wave_sync();
    if (i != kNone) {
      const uint64_t xa = load_aux(r.vals, i, B);
      WalkPlanner<B, H, EXT> Pl(g, r, L, cap);
      Pl.op = r.op_base + i;
      Pl.T = tab_of(g, r.op_table, r.tdesc, i);
      uint32_t h[H];
      hash_key<H, EXT>(g, Pl.T, x, h);
      uint32_t st;
      if (g.scheme == CK_RATTLE) st = Pl.rattle(x, xa);
      else if (g.scheme == CK_QUEUE) st = Pl.queue_kick(x, xa, h);
      else st = Pl.random_walk(x, xa, h);
      Pl.finish(i, st, win, &s_views);
    }
    wave_sync();
  }
  if (threadIdx.x == 0 && s_views) r.wg_views[blockIdx.x] += s_views;
}

// ---- breadth-first and sorted search (Sec. 5) ------------------------------
// Records are kept in runs: run r holds the B slots of the r-th bin put on
// the search frontier (runs 0..H-1 are the key's own bins, in hash order), so
// record e is slot e % B of run e / B.  A bin is visited iff it is the bin of
// a run (a viewed bin that is not terminal becomes a run; a terminal one ends
// the search).  When a run is created its B keys are hashed in parallel and
// each record's candidate bins (its key's other bins) are stored; the root
// records keep theirs in registers.  BFS expands records in index order;
// sorted search keeps 16 FIFO buckets of runs by spawn count and expands the
// head record of the lowest non-empty bucket.
//
// A wavefront runs 64 / W searches side by side, W lanes each (a group).  A
// search expands its frontier W / B bins at a time: the next records in
// search order are taken together, their candidate bins are fetched by one
// group-wide load (B lanes per bin), and the records are then processed one
// by one in order, exactly as the serial search does.  Searches read the
// round-start snapshot only, so fetching ahead changes no result; a group of
// records is abandoned at a record boundary when a new run has gone to a
// lower bucket, since the next record in order is then another one.  The
// first kSearchLdsRuns runs of a search live in LDS, the rest (long
// searches only) in workgroup scratch.
//
// The plan (chain moves root first, then the terminal write, preceded by the
// twin's mark clear when a ghost duplicate is replaced) goes straight to the
// workgroup's arena region, one move per lane.
constexpr uint32_t kRootParent = 0xFFFFFFFFu;
constexpr uint32_t kSearchLdsRuns = 128;
constexpr int kSearchW = 16;  // lanes per search
constexpr int kSearchLoads = 2;  // bin slots per lane in one group load
// BFS over bins of 8 slots or more loads twice as deep: FIFO order never
// abandons a fetched group (only the terminal bin ends one early), so deeper
// loads hide more latency, while the spawn-count orders would discard them
// whenever a new run goes to a lower bucket, and would spill registers.
constexpr int kSearchLoadsFifo8 = 4;

size_t search_runs(const Geo& g) { return (size_t)g.max_search + 8 + g.H; }
// search orders: BFS (FIFO), sorted search (spawn count), their hybrid
// (depth, then spawn count)
constexpr int kOrderFifo = 0, kOrderCount = 1, kOrderDepthCount = 2;
// Candidate words (a listed record's other bins) of one search kept in LDS;
// the rest (long searches only) go to workgroup scratch.
constexpr uint32_t kCandLds = 128;
// LDS words of one search group: run bins, parents and links (kSearchLdsRuns
// each), then bucket heads and tails, and the hybrid's next-depth heads and
// tails (16 each), then the first kCandLds candidate words.  The kernel's
// group stride and the launch's size both come from here.
__host__ __device__ constexpr uint32_t search_group_lds_words() {
  return 3 * kSearchLdsRuns + 4 * 16 + kCandLds;
}
static size_t search_group_scratch_bytes(const Geo& g) {
  const size_t RC = search_runs(g);
  return ((RC * g.B * (g.H - 1) + 5 * RC) * 4 + 255) & ~(size_t)255;
}

// At least four wavefronts per SIMD: the register budget that keeps 16
// one-wavefront workgroups resident per CU.
// EXT: the instance for upserts, stashes and biased hashes (the plain one has
// none of their branches, which would cost registers at this kernel's budget).
template <int B, int H, int O, bool EXT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_plan_search(
    Geo g, Round r) {
  constexpr int W = kSearchW;
  constexpr int P = 64 / W;       // searches per wavefront
  constexpr uint32_t C = H - 1;   // candidates per record
  // bin slots each lane loads per group load
  constexpr int KW = (B >= 8 && O == kOrderFifo) ? kSearchLoadsFifo8 : kSearchLoads;
  constexpr uint32_t G = KW * W / B;        // bins per group load
  constexpr int UW = (int)((G + W - 1) / W);  // group units per lane
  constexpr uint32_t RB = H * B;  // root records
  constexpr uint32_t RL = kSearchLdsRuns;
  constexpr int RBW = (int)((RB + W - 1) / W);  // root records per lane
  static_assert(G >= C, "search group too narrow");
  extern __shared__ uint32_t lds32[];
  __shared__ uint32_t win[4];  // arena region, spawn region
  __shared__ unsigned long long s_views;  // bins viewed by this workgroup's plans
  const int lane = threadIdx.x;
  const int gl = lane % W;            // lane within the group
  const int gb = lane - gl;           // the group's first lane
  const int gi = lane / W;            // group index
  const uint64_t gmask = W == 64 ? ~0ull : ((1ull << W) - 1);
  auto gballot = [&](bool p) -> uint64_t { return (__ballot(p) >> gb) & gmask; };
  const uint32_t RC = g.max_search + 8 + H;
  uint32_t* rbinL = lds32 + (size_t)gi * search_group_lds_words();
  uint32_t* rparL = rbinL + RL;
  uint32_t* rnextL = rparL + RL;
  uint32_t* bhead = rnextL + RL;  // record at the head of each bucket
  uint32_t* btail = bhead + 16;   // last run of each bucket
  uint32_t* nhead = btail + 16;   // the hybrid: the next depth's buckets
  uint32_t* ntail = nhead + 16;
  uint32_t* candL = ntail + 16;   // candidate words 0 .. kCandLds - 1
  static_assert(3 * RL + 4 * 16 + kCandLds <= search_group_lds_words(),
                "search group LDS layout");
  // the group's scratch: one workgroup-uniform base plus a per-group word
  // offset, so the arrays cost one register, not a pointer each
  uint32_t* const wsb = (uint32_t*)((char*)r.wg_scratch + (size_t)blockIdx.x * r.wg_scratch_bytes);
  const uint32_t go = (uint32_t)gi * (r.wg_scratch_bytes / P / 4);
  const uint32_t o_spl = RC * B * C;  // cand: RC * B * C words first
  const uint32_t o_path = o_spl + RC;
  const uint32_t o_rbin = o_path + RC;  // runs >= RL
  const uint32_t o_rpar = o_rbin + RC;
  const uint32_t o_rnext = o_rpar + RC;
  auto cand = [&](uint32_t j) -> uint32_t& { return j < kCandLds ? candL[j] : wsb[go + j]; };
  auto spl = [&](uint32_t j) -> uint32_t& { return wsb[go + o_spl + j]; };
  auto path = [&](uint32_t j) -> uint32_t& { return wsb[go + o_path + j]; };
  auto rbinG = [&](uint32_t j) -> uint32_t& { return wsb[go + o_rbin + j]; };
  auto rparG = [&](uint32_t j) -> uint32_t& { return wsb[go + o_rpar + j]; };
  auto rnextG = [&](uint32_t j) -> uint32_t& { return wsb[go + o_rnext + j]; };
  auto rbin_at = [&](uint32_t j) -> uint32_t { return j < RL ? rbinL[j] : rbinG(j); };
  auto rpar_at = [&](uint32_t j) -> uint32_t { return j < RL ? rparL[j] : rparG(j); };
  auto rnext_at = [&](uint32_t j) -> uint32_t { return j < RL ? rnextL[j] : rnextG(j); };
  auto set_run = [&](uint32_t j, uint32_t bin, uint32_t par) {  // group leader
    if (j < RL) { rbinL[j] = bin; rparL[j] = par; }
    else { rbinG(j) = bin; rparG(j) = par; }
  };
  auto set_next = [&](uint32_t j, uint32_t nx) {  // group leader
    if (j < RL) rnextL[j] = nx;
    else rnextG(j) = nx;
  };
  // spawn counts order the search (sorted search, the hybrid); the hybrid
  // spawns a whole depth before the next
  constexpr bool by_count = O != kOrderFifo;
  constexpr bool hybrid = O == kOrderDepthCount;
  const bool need_meta = by_count || g.ghost;
  // k-at-a-time spawning (two-choice bins of 4 or 8 slots): a group is the
  // next spawn_k records in search order, across buckets, all spawned
  constexpr bool kable = C == 1 && B >= 4 && !hybrid;
  const bool kmode = kable && g.spawn_k > 1;
  const uint32_t glim = kmode ? g.spawn_k * C : G;  // units of one group
  if (lane == 0) {
    region_init(win, r.arena_cap);
    region_init(win + 2, r.spawn_cap);
    s_views = 0;
  }
  wave_sync();
  EvictWork Wk;
  Wk.init(r, 64 / fresh_lanes(B));
  // the group's op of batch kb is item kb + gi; item() is wave-uniform
  auto batch_item = [&](uint32_t kb) -> uint32_t {
    uint32_t mine = kNone;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint32_t v = Wk.item(kb + (uint32_t)p);
      if (gi == p) mine = v;
    }
    return mine;
  };

  // Ops are software-pipelined: while batch kb is planned, the next batch's
  // ops and keys are in flight, and their root bins are fetched as soon as
  // the current searches end.
  uint32_t i_nx = batch_item(0);
  uint64_t x_nx = 0;
  Tab T_nx{0u, 0u};
  uint32_t h_nx[H];
#pragma unroll
  for (int j = 0; j < H; ++j) h_nx[j] = 0;
  // next op's root slots: root record e = gl + s W in lane gl, slot s
  uint64_t rk_nx[RBW];
  uint32_t rm_nx[RBW];  // their bins' metadata words (spawn-count orders)
#pragma unroll
  for (int t = 0; t < RBW; ++t) { rk_nx[t] = kEmpty; rm_nx[t] = 0; }
  auto fetch_roots = [&]() {
    if (i_nx == kNone) return;
    T_nx = tab_of(g, r.op_table, r.tdesc, i_nx);
    hash_key<H, EXT>(g, T_nx, x_nx, h_nx);
#pragma unroll
    for (int t = 0; t < RBW; ++t) {
      const int e = gl + t * W;
      if (e < (int)RB) {
        const int q = e / B, sl = e % B;
        uint32_t hb = h_nx[0];
#pragma unroll
        for (int j = 1; j < H; ++j)
          if (q == j) hb = h_nx[j];
        rk_nx[t] = g.slots[(uint64_t)hb * B + sl].x;
        if (by_count) rm_nx[t] = g.meta[hb];
      }
    }
  };
  if (i_nx != kNone) x_nx = r.keys[i_nx];
  fetch_roots();
  for (uint32_t kb = 0;; kb += P) {
    if (__ballot(i_nx != kNone) == 0) break;  // wave-uniform
    const uint32_t i = i_nx;
    const bool have = i != kNone;
    const Tab T = T_nx;
    uint32_t h[H];
#pragma unroll
    for (int j = 0; j < H; ++j) h[j] = h_nx[j];
    uint64_t rkey[RBW];
    uint32_t rmeta[RBW];
#pragma unroll
    for (int t = 0; t < RBW; ++t) { rkey[t] = rk_nx[t]; rmeta[t] = rm_nx[t]; }
    i_nx = batch_item(kb + P);
    if (i_nx != kNone) x_nx = r.keys[i_nx];
    // ops reach this planner after the fresh planner found no room in the
    // same snapshot: first fit viewed all H bins, ghost inserts both bins
    uint32_t views = g.ghost ? 2u : (uint32_t)H;
    // ---- root runs: the key's own bins (slots already fetched, H*B lanes)
    uint32_t rc[RBW][C];  // root record e's candidates: lane e % W, rc[e / W]
    uint32_t bk[RBW];
#pragma unroll
    for (int t2 = 0; t2 < RBW; ++t2) {
      bk[t2] = 0;
#pragma unroll
      for (int j = 0; j < (int)C; ++j) rc[t2][j] = 0;
      const int e = gl + t2 * W;
      if (have && e < (int)RB) {
        const int q = e / B;
        uint32_t hb = h[0];
#pragma unroll
        for (int j = 1; j < H; ++j)
          if (q == j) hb = h[j];
        if (by_count) bk[t2] = min(15u, (rmeta[t2] >> 8) & 0xFu);
        uint32_t hv[H];
        hash_key<H, EXT>(g, T, rkey[t2], hv);
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
          if (hv[j] == hb) continue;
#pragma unroll
          for (int t = 0; t < (int)C; ++t)
            if (t == (int)o) rc[t2][t] = hv[j];
          ++o;
        }
      }
    }
    if (have && gl < H) {
      uint32_t hb = h[0];
#pragma unroll
      for (int j = 1; j < H; ++j)
        if (gl == j) hb = h[j];
      rbinL[gl] = hb;
      rparL[gl] = kRootParent;
    }
    for (int j = gl; j < 16; j += W) {
      bhead[j] = kNone;
      btail[j] = kNone;
      nhead[j] = kNone;
      ntail[j] = kNone;
    }
    uint32_t bks[H];  // root run j's bucket: from root record j B
#pragma unroll
    for (int j = 0; j < H; ++j) {
      uint32_t v = 0;
#pragma unroll
      for (int t2 = 0; t2 < RBW; ++t2) {
        const uint32_t u = __shfl(bk[t2], gb + (j * B) % W, 64);
        if (t2 == (j * B) / W) v = u;
      }
      bks[j] = v;
    }
    wave_sync();
    uint32_t bmask = 0;   // spawn-count orders: non-empty buckets (group-uniform)
    uint32_t nbmask = 0;  // the hybrid: non-empty buckets of the next depth
    if (have && by_count) {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        if (gl == 0) {
          rnextL[j] = kNone;
          if (btail[bks[j]] == kNone) bhead[bks[j]] = j * B;
          else set_next(btail[bks[j]], j);
          btail[bks[j]] = j;
        }
        bmask |= 1u << bks[j];
      }
    }
    wave_sync();
    uint32_t nruns = H;
    uint32_t head = 0;  // BFS: next record
    uint32_t nsp = 0;
    bool found = false;
    uint32_t term_e = 0, term_c = 0;
    uint64_t tkey = kEmpty;  // the terminal bin's view (group lanes < B)
    uint32_t tmeta = 0;
    bool done = !have;
    while (!done) {
      // ---- the next records in search order, as one group; unit u (a
      // record and one of its candidates) lives in lane u % W, register u / W
      uint32_t my_e[UW], my_j[UW];
#pragma unroll
      for (int t = 0; t < UW; ++t) { my_e[t] = 0; my_j[t] = 0; }
      uint32_t nu = 0;
      if (!by_count) {
        const uint32_t tail = nruns * B;
        if (head == tail) break;
        const uint32_t nrec = min(glim / C, tail - head);
        nu = nrec * C;
#pragma unroll
        for (int t = 0; t < UW; ++t) {
          const uint32_t u = (uint32_t)(gl + t * W);
          my_e[t] = head + u / C;
          my_j[t] = u % C;
        }
      } else {
        if (bmask == 0) {
          if (!hybrid || nbmask == 0) break;
          // the hybrid: this depth is spawned out, the next one's buckets
          // become current
          wave_sync();
          if (gl < 16) {
            bhead[gl] = nhead[gl];
            btail[gl] = ntail[gl];
            nhead[gl] = kNone;
            ntail[gl] = kNone;
          }
          wave_sync();
          bmask = nbmask;
          nbmask = 0;
        }
        int kb2 = __ffs(bmask) - 1;
        uint32_t e = bhead[kb2];
        uint32_t bm = bmask;
        for (;;) {
          if (e == kNone) {  // k at a time: on to the next bucket
            if (!kmode) break;
            bm &= ~(1u << kb2);
            if (bm == 0) break;
            kb2 = __ffs(bm) - 1;
            e = bhead[kb2];
            continue;
          }
          if (nu + C > glim) break;
#pragma unroll
          for (uint32_t j = 0; j < C; ++j)
#pragma unroll
            for (int t = 0; t < UW; ++t)
              if ((uint32_t)(gl + t * W) == nu + j) { my_e[t] = e; my_j[t] = j; }
          nu += C;
          if (((e + 1) & (B - 1)) != 0) {
            e = e + 1;
          } else {
            const uint32_t nr = rnext_at(e / B);
            e = nr == kNone ? kNone : nr * B;
          }
        }
      }
      // ---- candidate bins (root records from registers), then contents
      uint32_t cu[UW];
#pragma unroll
      for (int t = 0; t < UW; ++t) {
        uint32_t rv = 0;
#pragma unroll
        for (int t2 = 0; t2 < RBW; ++t2) {
#pragma unroll
          for (int tc = 0; tc < (int)C; ++tc) {
            const uint32_t v = __shfl(rc[t2][tc], gb + (int)(my_e[t] % W), 64);
            if ((uint32_t)tc == my_j[t] && my_e[t] / W == (uint32_t)t2) rv = v;
          }
        }
        cu[t] = 0;
        if ((uint32_t)(gl + t * W) < nu)
          cu[t] = my_e[t] < RB ? rv : cand(my_e[t] * C + my_j[t]);
      }
      // load k: lane gl reads slot p % B of unit p / B, p = k W + gl
      ulonglong2 sv[KW];
      uint32_t mv[KW];
#pragma unroll
      for (int k = 0; k < KW; ++k) {
        const uint32_t pidx = (uint32_t)(k * W + gl);
        const uint32_t pu = pidx / B, ps = pidx % B;
        const uint32_t cb = __shfl(cu[(k * W) / (B * W)], gb + (int)(pu % W), 64);
        sv[k] = make_ulonglong2(kEmpty, 0ull);
        mv[k] = 0;
        if (pu < nu) {
          sv[k] = g.slots[(uint64_t)cb * B + ps];
          if (need_meta) mv[k] = g.meta[cb];
        }
      }
      if constexpr (C == 1 && B >= 4) {
        // ---- the whole group at once (one candidate per record, at most one
        // record per lane): the serial rules become a cut in record order.
        static_assert(G <= (uint32_t)W, "one record per lane");
        const uint32_t u = (uint32_t)gl;  // this lane's record in the group
        const bool valid = u < nu;
        const uint32_t e_u = my_e[0], c_u = cu[0];
        // visited: a run's bin, or the candidate of an earlier record
        bool seen = false;
        const uint32_t nl = min(nruns, RL);
        for (uint32_t j = 0; j < nl; ++j) seen |= rbinL[j] == c_u;
        for (uint32_t j = RL; j < nruns; ++j) seen |= rbinG(j) == c_u;
#pragma unroll
        for (uint32_t v = 0; v < G; ++v) {
          const uint32_t cv = __shfl(c_u, gb + (int)v, 64);
          seen |= v < u && v < nu && cv == c_u;
        }
        const bool nv = valid && !seen;
        // terminal bins: a ballot per load; record u's slots are bits
        // (u B) % W .. + B - 1 of load (u B) / W
        uint64_t tb[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) {
          const uint32_t pidx = (uint32_t)(k * W + gl);
          const uint32_t pu = pidx / B, ps = pidx % B;
          tb[k] = gballot(pu < nu && (sv[k].x == kEmpty || (g.ghost && ((mv[k] >> ps) & 1u))));
        }
        const uint32_t ku = (u * B) / W, su = (u * B) % W;
        uint64_t tbu = 0;
        uint32_t mu = 0;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
          const uint32_t m2 = __shfl(mv[k], gb + (int)su, 64);
          if (ku == (uint32_t)k) { tbu = tb[k]; mu = m2; }
        }
        const bool term = ((tbu >> su) & ((1ull << B) - 1)) != 0;
        const uint32_t b2 = min(15u, (mu >> 8) & 0xFu);
        // the cut: first terminal (kept), first run into a lower bucket
        // (kept, then regroup), or the view that would pass max_search (not kept)
        const uint32_t kb_now = by_count ? (uint32_t)(__ffs(bmask) - 1) : 0u;
        const uint64_t NV = gballot(nv);
        const uint64_t below = (1ull << u) - 1;
        const uint32_t rank = (uint32_t)__popcll(NV & below);
        const uint32_t avail = g.max_search - views;
        const uint64_t TERM = gballot(nv && term);
        // (the hybrid's new runs are one depth down: never ahead of this group)
        const uint64_t LOW =
            (by_count && !hybrid && !kmode) ? gballot(nv && !term && b2 < kb_now) : 0ull;
        const uint64_t CAP = gballot(nv && rank == avail);
        const uint32_t t_term = TERM ? (uint32_t)__ffsll((unsigned long long)TERM) - 1 : 64u;
        const uint32_t t_low = LOW ? (uint32_t)__ffsll((unsigned long long)LOW) - 1 : 64u;
        const uint32_t t_cap = CAP ? (uint32_t)__ffsll((unsigned long long)CAP) - 1 : 64u;
        uint32_t cut = nu;
        bool capped = false;
        if (kmode) {
          // spawned together: every record of the group views its candidate
          // (up to the cap); the first bin with room among them ends the chain
          if (t_cap < 64u) cut = t_cap;
          found = t_term < cut;
          capped = t_cap < 64u && !found;
        } else if (t_cap <= t_term && t_cap <= t_low && t_cap < 64u) {
          cut = t_cap;
          capped = true;
        } else if (t_term < t_low) {
          cut = t_term + 1;
          found = true;
        } else if (t_low < 64u) {
          cut = t_low + 1;
        }
        const uint64_t upto = cut >= 64 ? ~0ull : ((1ull << cut) - 1);
        const uint64_t VIEW = NV & upto;
        const uint64_t RUNS = VIEW & ~TERM;
        views += (uint32_t)__popcll(VIEW);
        // spawn list (spawn-count orders): every record that viewed its candidate
        if (by_count && ((VIEW >> u) & 1ull)) spl(nsp + (uint32_t)__popcll(VIEW & below)) = e_u / B;
        if (by_count) nsp += (uint32_t)__popcll(VIEW);
        // new runs, in record order
        const bool mkrun = (RUNS >> u) & 1ull;
        const uint32_t run_u = nruns + (uint32_t)__popcll(RUNS & below);
        if (mkrun) set_run(run_u, c_u, e_u);
#pragma unroll
        for (int k = 0; k < KW; ++k) {
          const uint32_t pidx = (uint32_t)(k * W + gl);
          const uint32_t pu = pidx / B, ps = pidx % B;
          const uint32_t rp = __shfl(run_u, gb + (int)(pu % W), 64);
          const uint32_t cp = __shfl(c_u, gb + (int)(pu % W), 64);
          if (pu < G && ((RUNS >> pu) & 1ull)) {
            uint32_t hv[H];
            hash_key<H, EXT>(g, T, sv[k].x, hv);
            cand(rp * B + ps) = hv[0] == cp ? hv[1] : hv[0];
          }
        }
        const uint32_t nnew = (uint32_t)__popcll(RUNS);
        if (found) {
          term_e = __shfl(e_u, gb + (int)t_term, 64);
          term_c = __shfl(c_u, gb + (int)t_term, 64);
          const uint32_t kt = (t_term * B) / W, st2 = (t_term * B) % W;
#pragma unroll
          for (int k = 0; k < KW; ++k) {
            const uint64_t a = __shfl(sv[k].x, gb + (int)(st2 + ((uint32_t)gl & (B - 1))), 64);
            const uint32_t m2 = __shfl(mv[k], gb + (int)st2, 64);
            if (kt == (uint32_t)k) { tkey = a; tmeta = m2; }
          }
        }
        // pop the processed records, then link the new runs
        if (!by_count) {
          head += cut;
        } else {
          // the group's records leave the front of the buckets: the first
          // `cut` records of the lowest bucket, or (k at a time, when the
          // search goes on) all nu records, lowest bucket first
          uint32_t left = kmode ? ((found || capped) ? 0u : nu) : cut;
          bool first_pass = true;
          while (left || first_pass) {
            first_pass = false;
            const uint32_t kbp = kmode ? (uint32_t)(__ffs(bmask) - 1) : kb_now;
            if (kmode && bmask == 0) break;
            uint32_t eh = bhead[kbp];
            for (; left && eh != kNone; --left) {
              if (((eh + 1) & (B - 1)) != 0) {
                eh = eh + 1;
              } else {
                const uint32_t nr = rnext_at(eh / B);
                eh = nr == kNone ? kNone : nr * B;
              }
            }
            wave_sync();
            if (gl == 0) {
              bhead[kbp] = eh;
              if (eh == kNone) btail[kbp] = kNone;
            }
            if (eh == kNone) bmask &= ~(1u << kbp);
            wave_sync();
            if (!kmode) break;
          }
          uint64_t rr = RUNS;
          while (rr) {
            const uint32_t v = (uint32_t)__ffsll((unsigned long long)rr) - 1;
            rr &= rr - 1;
            const uint32_t run = __shfl(run_u, gb + (int)v, 64);
            const uint32_t bv = __shfl(b2, gb + (int)v, 64);
            uint32_t* const lh = hybrid ? nhead : bhead;
            uint32_t* const lt = hybrid ? ntail : btail;
            if (gl == 0) {
              set_next(run, kNone);
              if (lt[bv] == kNone) lh[bv] = run * B;
              else set_next(lt[bv], run);
              lt[bv] = run;
            }
            if (hybrid) nbmask |= 1u << bv;
            else bmask |= 1u << bv;
            wave_sync();
          }
        }
        nruns += nnew;
        wave_sync();
        if (found || capped) done = true;
      } else {
      // ---- records one by one, in order
      for (uint32_t u = 0; u < nu && !done; u += C) {
        uint32_t e = 0;
#pragma unroll
        for (int t = 0; t < UW; ++t) {
          const uint32_t v = __shfl(my_e[t], gb + (int)(u % W), 64);
          if (u / W == (uint32_t)t) e = v;
        }
        if (by_count) {
          const int kb2 = bmask ? __ffs(bmask) - 1 : -1;
          if (kb2 < 0 || bhead[kb2] != e) break;  // order changed: regroup
          wave_sync();
          bool emptied = false;
          if (((e + 1) & (B - 1)) == 0) emptied = rnext_at(e / B) == kNone;
          if (gl == 0) {
            if (((e + 1) & (B - 1)) != 0) {
              bhead[kb2] = e + 1;
            } else {
              const uint32_t nr = rnext_at(e / B);
              bhead[kb2] = nr == kNone ? kNone : nr * B;
              if (nr == kNone) btail[kb2] = kNone;
            }
          }
          if (emptied) bmask &= ~(1u << kb2);
          wave_sync();
        } else {
          ++head;
        }
        bool spawned = false;
        for (uint32_t j = 0; j < C; ++j) {
          const uint32_t uu = u + j;
          uint32_t c = 0;
#pragma unroll
          for (int t = 0; t < UW; ++t) {
            const uint32_t v = __shfl(cu[t], gb + (int)(uu % W), 64);
            if (uu / W == (uint32_t)t) c = v;
          }
          bool seen = false;
          for (uint32_t base = 0; base < nruns; base += W) {
            const uint32_t q = base + (uint32_t)gl;
            seen |= gballot(q < nruns && rbin_at(q) == c) != 0;
          }
          if (seen) continue;
          if (views == g.max_search) { done = true; break; }
          if (by_count && !spawned) {
            if (gl == 0) spl(nsp) = e / B;
            ++nsp;
          }
          spawned = true;
          ++views;
          // unit uu's bin: slot sl in lane (uu B) % W + sl, load (uu B) / W
          const uint32_t kk = (uu * B) / W;
          const int src = gb + (int)((uu * B) % W + ((uint32_t)gl & (B - 1)));
          uint64_t vk = kEmpty;
          uint32_t vm = 0;
#pragma unroll
          for (int k = 0; k < KW; ++k) {
            const uint64_t a = __shfl(sv[k].x, src, 64);
            const uint32_t m2 = __shfl(mv[k], gb + (int)((uu * B) % W), 64);
            if (kk == (uint32_t)k) { vk = a; vm = m2; }
          }
          const bool empty = gl < B && vk == kEmpty;
          const bool dup = g.ghost && gl < B && vk != kEmpty && ((vm >> gl) & 1u);
          if (gballot(empty || dup) != 0) {
            found = true;
            term_e = e;
            term_c = c;
            tkey = vk;
            tmeta = vm;
            done = true;
            break;
          }
          // a new run: its records' candidate bins, its bin and parent
          const uint32_t run = nruns++;
          if (gl < B) {
            uint32_t hv[H];
            hash_key<H, EXT>(g, T, vk, hv);
            uint32_t o = 0;
#pragma unroll
            for (int q = 0; q < H; ++q)
              if (hv[q] != c) cand((run * B + gl) * C + o++) = hv[q];
          }
          if (gl == 0) set_run(run, c, e);
          wave_sync();
          if (by_count) {
            const uint32_t b2 = min(15u, (vm >> 8) & 0xFu);
            uint32_t* const lh = hybrid ? nhead : bhead;
            uint32_t* const lt = hybrid ? ntail : btail;
            if (gl == 0) {
              set_next(run, kNone);
              if (lt[b2] == kNone) lh[b2] = run * B;
              else set_next(lt[b2], run);
              lt[b2] = run;
            }
            if (hybrid) nbmask |= 1u << b2;
            else bmask |= 1u << b2;
            wave_sync();
          }
        }
      }
      }
    }
    fetch_roots();
    // ---- spawn counts go to the spawn arena for every plan, winning or not
    uint32_t soff = 0;
    if (by_count && nsp > 0) {
      uint32_t o = 0;
      if (gl == 0) o = region_take(win + 2, nsp, r.ctr);
      soff = __shfl(o, gb, 64);
      if (soff != kNone)
        for (uint32_t j = gl; j < nsp; j += W) r.spawns[soff + j] = rbin_at(spl(j));
      else
        nsp = 0;
    }
    // ---- the plan
    uint32_t nm = 0, depth = 0, twin = 0, off = 0;
    if (found) {
      // path: term_e, its parent record, ..., a root record
      uint32_t preg = 0;
      for (uint32_t cur = term_e;;) {
        if (gl == (int)depth) preg = cur;
        if (gl == 0) path(depth) = cur;
        ++depth;
        const uint32_t par = rpar_at(cur / B);
        if (par == kRootParent) break;
        cur = par;
      }
      const uint32_t emask = (uint32_t)(gballot(gl < B && tkey == kEmpty) & ((1ull << B) - 1));
      uint32_t tslot;
      uint64_t dk = 0;
      if (emask) {
        tslot = ffs32(emask);
      } else {
        const uint32_t dmask = (uint32_t)(gballot(gl < B && tkey != kEmpty &&
                                                  ((tmeta >> gl) & 1u)) & ((1ull << B) - 1));
        tslot = ffs32(dmask);
        dk = __shfl(tkey, gb + (int)tslot, 64);
        twin = 1;
      }
      nm = depth + 1 + twin;
      uint32_t o = 0;
      if (gl == 0) o = region_take(win, nm, r.ctr);
      off = __shfl(o, gb, 64);
      wave_sync();  // the path array, written by the group leader
      // the terminal write's content is the deepest record's snapshot content
      const ulonglong2 tv = g.slots[(uint64_t)rbin_at(term_e / B) * B + term_e % B];
      uint32_t tb = 0, tws = 0;
      if (twin) {  // the duplicate's twin, in the duplicate key's other bin
        uint32_t hd[2];
        hash_key<2, EXT>(g, T, dk, hd);
        tb = hd[0] == term_c ? hd[1] : hd[0];
        uint64_t tk2 = kEmpty;
        if (gl < B) tk2 = g.slots[(uint64_t)tb * B + gl].x;
        tws = ffs32((uint32_t)(gballot(gl < B && tk2 == dk) & ((1ull << B) - 1)));
      }
      // chain moves: move m puts the content of path[depth - m] (x for m = 0)
      // into the slot of path[depth - 1 - m]
      for (uint32_t mb = 0; mb < depth; mb += W) {
        const uint32_t m = mb + (uint32_t)gl;
        const uint32_t d = m < depth ? depth - 1 - m : 0;
        const uint32_t p_reg = __shfl(preg, gb + (int)min(d, (uint32_t)W - 1), 64);
        const uint32_t s_reg = __shfl(preg, gb + (int)min(d + 1, (uint32_t)W - 1), 64);
        if (m < depth) {
          const uint32_t prec = depth <= (uint32_t)W ? p_reg : path(d);
          Move mvv;
          if (m == 0) {  // the op's own key and value (re-read: not kept live)
            mvv.key = r.keys[i];
            mvv.aux = load_aux(r.vals, i, B);
          } else {
            const uint32_t srec = depth <= (uint32_t)W ? s_reg : path(d + 1);
            const ulonglong2 v = g.slots[(uint64_t)rbin_at(srec / B) * B + srec % B];
            mvv.key = v.x;
            mvv.aux = v.y;
          }
          mvv.bin = rbin_at(prec / B);
          mvv.slot = (uint8_t)(prec % B);
          mvv.flags = 0;
          mvv.pad = 0;
          if (off != kNone) {
            r.arena[off + m] = mvv;
            claim(g, r, mvv.bin, i);
          }
        }
      }
      if (gl == 0 && off != kNone) {
        if (twin) {
          Move t2;
          t2.key = 0;
          t2.aux = 0;
          t2.bin = tb;
          t2.slot = (uint8_t)tws;
          t2.flags = MV_DUPCLR;
          t2.pad = 0;
          r.arena[off + depth] = t2;
          claim(g, r, tb, i);
        }
        Move t1;
        t1.key = tv.x;
        t1.aux = tv.y;
        t1.bin = term_c;
        t1.slot = (uint8_t)tslot;
        t1.flags = 0;
        t1.pad = 0;
        r.arena[off + depth + twin] = t1;
        claim(g, r, term_c, i);
      }
    }
    if (have && gl == 0) {
      // a failed search's key goes to the stash if it has room
      const uint32_t se = (EXT && !found) ? stash_take(g, r, i) : kNone;
      r.hdr[i] = make_uint4(
          hdr_pack(found ? PL_OK : (se != kNone ? PL_STASHED : PL_FAIL), twin, nm) | kHdrArena |
              ((EXT && r.upsert) ? kHdrKeyClaim : 0u) | (se != kNone ? kHdrStash : 0u),
          views + ((EXT && r.upsert) ? (uint32_t)H + (g.stash_n ? 1u : 0u) : 0u), off,
          found ? depth : (se != kNone ? se : 0u));
      r.hdr_spawn[i] = make_uint2(nsp, soff);
      atomicAdd(&s_views, (unsigned long long)views);
    }
    wave_sync();
  }
  if (threadIdx.x == 0 && s_views) r.wg_views[blockIdx.x] += s_views;
}

static bool is_search(uint32_t scheme) {
  return scheme == CK_BFS || scheme == CK_SORTED || scheme == CK_HYBRID;
}

size_t evict_lds_bytes(const Geo& g) {
  if (is_search(g.scheme))
    return (64 / kSearchW) * search_group_lds_words() * 4 + 64;
  return (64 / kWalkW) * walk_group_lds_bytes(g) + 64;
}

size_t evict_wg_scratch_bytes(const Geo& g) {
  if (is_search(g.scheme))
    return (64 / kSearchW) * search_group_scratch_bytes(g);
  return (64 / kWalkW) * walk_group_scratch_bytes(g);
}

// Workgroups of a launch after a sub-batch's first round, whose pending count
// is known only on the device: enough to fill the device, each taking as
// many passes as the count needs.
constexpr uint32_t kTailPlanBlocks = 2048;

// Rounds that need the extended kernel instances: upserts, a stash (inserts,
// deletes and overwrites search or fill it), or biased hashes.
static bool extended(const Geo& g, const Round& r) {
  return r.upsert || g.stash_n || g.hash_bias;
}
constexpr uint32_t kTailCommitBlocks = 1024;

template <int B, int H>
static void evict_go(const Geo& g, const Round& r, uint32_t grid, hipStream_t s) {
  const size_t lds = evict_lds_bytes(g);
  if (extended(g, r) && !is_search(g.scheme)) {
    hipLaunchKernelGGL((k_plan_walk<B, H, true>), dim3(grid), dim3(64), lds, s, g, r);
  } else if (extended(g, r)) {
    if (g.scheme == CK_BFS)
      hipLaunchKernelGGL((k_plan_search<B, H, kOrderFifo, true>), dim3(grid), dim3(64), lds, s,
                         g, r);
    else if (g.scheme == CK_SORTED)
      hipLaunchKernelGGL((k_plan_search<B, H, kOrderCount, true>), dim3(grid), dim3(64), lds, s,
                         g, r);
    else
      hipLaunchKernelGGL((k_plan_search<B, H, kOrderDepthCount, true>), dim3(grid), dim3(64), lds,
                         s, g, r);
  } else if (g.scheme == CK_BFS)
    hipLaunchKernelGGL((k_plan_search<B, H, kOrderFifo, false>), dim3(grid), dim3(64), lds, s, g,
                       r);
  else if (g.scheme == CK_SORTED)
    hipLaunchKernelGGL((k_plan_search<B, H, kOrderCount, false>), dim3(grid), dim3(64), lds, s, g,
                       r);
  else if (g.scheme == CK_HYBRID)
    hipLaunchKernelGGL((k_plan_search<B, H, kOrderDepthCount, false>), dim3(grid), dim3(64), lds,
                       s, g, r);
  else
    hipLaunchKernelGGL((k_plan_walk<B, H, false>), dim3(grid), dim3(64), lds, s, g, r);
}

template <int B, int H>
static void fresh_go(const Geo& g, const Round& r, hipStream_t s) {
  const uint64_t threads = (uint64_t)r.npend * fresh_lanes(B);
  uint32_t grid = (uint32_t)((threads + 255) / 256);
  if (!r.first) grid = std::min(grid, kTailPlanBlocks);
  if (extended(g, r)) hipLaunchKernelGGL((k_plan_fresh<B, H, true>), dim3(grid), dim3(256), 0, s, g, r);
  else hipLaunchKernelGGL((k_plan_fresh<B, H, false>), dim3(grid), dim3(256), 0, s, g, r);
}

#define CK_DISPATCH(FN, ...)                                  \
  switch (g.B) {                                              \
    case 1:                                                   \
      if (g.H == 2) FN<1, 2>(__VA_ARGS__);                    \
      else if (g.H == 3) FN<1, 3>(__VA_ARGS__);               \
      else FN<1, 4>(__VA_ARGS__);                             \
      break;                                                  \
    case 2: FN<2, 2>(__VA_ARGS__); break;                     \
    case 4: FN<4, 2>(__VA_ARGS__); break;                     \
    case 8: FN<8, 2>(__VA_ARGS__); break;                     \
    default: return hipErrorInvalidValue;                     \
  }

template <int B, int H>
static void evict_occupancy(const Geo& g, int* per_cu) {
  const size_t lds = evict_lds_bytes(g);
  // the plain instances (the extended ones have the same launch bounds)
  if (g.scheme == CK_BFS)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, k_plan_search<B, H, kOrderFifo, false>, 64, lds);
  else if (g.scheme == CK_SORTED)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, k_plan_search<B, H, kOrderCount, false>, 64, lds);
  else if (g.scheme == CK_HYBRID)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, k_plan_search<B, H, kOrderDepthCount, false>, 64, lds);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_plan_walk<B, H, false>, 64, lds);
}

// Eviction-planner workgroups that can be resident on one compute unit at
// once (registers, LDS and wave slots all counted).
int evict_resident_per_cu(const Geo& g) {
  int per_cu = 0;
  auto go = [&]() -> hipError_t {
    CK_DISPATCH(evict_occupancy, g, &per_cu);
    return hipSuccess;
  };
  if (go() != hipSuccess) return 0;
  return per_cu;
}

hipError_t launch_plan_fresh(const Geo& g, const Round& r, hipStream_t s) {
  if (r.npend == 0) return hipSuccess;
  CK_DISPATCH(fresh_go, g, r, s);
  return hipGetLastError();
}

hipError_t launch_plan_evict(const Geo& g, const Round& r, uint32_t grid, hipStream_t s) {
  if (r.npend == 0) return hipSuccess;
  CK_DISPATCH(evict_go, g, r, grid, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// delete planning: B lanes per op
// ---------------------------------------------------------------------------
template <int B, int H>
__device__ __forceinline__ void delete_one(const Geo& g, const Round& r, const GroupCtx<B>& G,
                                           uint32_t i) {
  if (r.first && G.sl == 0) zero_op_counters(r, i);
  const uint64_t x = r.keys[i];
  const bool leader = G.sl == 0;
  uint32_t mb[2], ms[2];
  uint32_t nm = 0, probes = 0, se = kNone;
  uint32_t status = PL_NOTFOUND;
  if (x != kEmpty) {
    uint32_t h[H];
    hash_key<H>(g, tab_of(g, r.op_table, r.tdesc, i), x, h);
#pragma unroll
    for (int hi = 0; hi < H; ++hi) {
      ulonglong2 s = g.slots[(uint64_t)h[hi] * B + G.sl];
      ++probes;
      const uint32_t m = G.ballot(s.x == x);
      if (m) {
        const uint32_t slot = ffs32(m);
        mb[nm] = h[hi];
        ms[nm] = slot;
        ++nm;
        if (g.ghost && ((g.meta[h[hi]] >> slot) & 1u)) {
          const uint32_t tb = h[1 - hi];
          ulonglong2 t = g.slots[(uint64_t)tb * B + G.sl];
          ++probes;
          const uint32_t tm = G.ballot(t.x == x);
          mb[nm] = tb;
          ms[nm] = ffs32(tm);
          ++nm;
        }
        status = PL_OK;
        break;
      }
    }
    if (status == PL_NOTFOUND && g.stash_n) {  // then the stash, one more probe
      ++probes;
      se = stash_find(g, table_of(r.op_table, i), x, G.sl, B,
                      [&](bool p) { return (uint64_t)G.ballot(p); });
      if (se != kNone) status = PL_OK;
    }
  }
  if (!leader) return;
  const uint32_t fl = r.overwrite ? MV_VALUE : MV_CLEAR;
  r.hdr[i] = make_uint4(
      hdr_pack(x == kEmpty ? PL_FAIL : status, 0, nm) | (se != kNone ? kHdrStash : 0u), probes,
      nm > 0 ? mb[0] : 0u, nm > 0 ? (ms[0] | (fl << 8)) : (se != kNone ? se : 0u));
  if (se != kNone) atomicMin(&g.stash_owner[se], r.tag | (unsigned long long)i);
  if (nm > 0) claim(g, r, mb[0], i);
  if (nm > 1) {
    r.imv[(size_t)i * kExtraInline] = IMove{mb[1], ms[1] | (fl << 8)};
    claim(g, r, mb[1], i);
  }
}

template <int B, int H>
__global__ __launch_bounds__(256) void k_plan_delete(Geo g, Round r) {
  GroupCtx<B> G;
  G.lane = threadIdx.x & 63;
  G.sl = G.lane % B;
  G.gshift = G.lane - G.sl;
  if (blockIdx.x == 0) round_start(r);
  Pending P;
  P.init(r);
  constexpr uint32_t opb = 256 / B;
  const uint32_t passes = (P.n + opb - 1) / opb;
  for (uint32_t c = blockIdx.x; c < passes; c += gridDim.x) {
    const uint32_t i = P.at(c * opb + threadIdx.x / B);
    if (i != kNone) delete_one<B, H>(g, r, G, i);
  }
}

template <int B, int H>
static void delete_go(const Geo& g, const Round& r, hipStream_t s) {
  const uint64_t threads = (uint64_t)r.npend * B;
  uint32_t grid = (uint32_t)((threads + 255) / 256);
  if (!r.first) grid = std::min(grid, kTailPlanBlocks);
  hipLaunchKernelGGL((k_plan_delete<B, H>), dim3(grid), dim3(256), 0, s, g, r);
}

hipError_t launch_plan_delete(const Geo& g, const Round& r, hipStream_t s) {
  if (r.npend == 0) return hipSuccess;
  CK_DISPATCH(delete_go, g, r, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// commit: kCommitLanes lanes per plan
// ---------------------------------------------------------------------------
// Spawn counts (Sec. 5) of one plan: +1 for each listed bin, saturating at
// 15.  One returning add per increment, four in flight per lane; an add that
// found the count already at 15 or more is taken back.  While the kernel
// runs the field may read above 15 (even carry into the byte above it,
// which only queue-kicking's hit counter uses, and queue-kicking keeps no
// spawn counts), but the adds that are kept never take it past 15 and every
// other add is undone, so when the kernel ends the field holds
// min(15, before + increments) whatever the interleaving.  Nothing reads the
// spawn counts during the commit kernel.
__device__ __forceinline__ void sc_increments(uint32_t* meta, const uint32_t* bins, uint32_t n,
                                              uint32_t first, uint32_t step) {
  for (uint32_t j0 = first; j0 < n; j0 += 4 * step) {
    uint32_t b[4], old[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t j = j0 + (uint32_t)u * step;
      b[u] = j < n ? bins[j] : kNone;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b[u] != kNone) old[u] = atomicAdd(meta + b[u], 1u << 8);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (b[u] != kNone && (old[u] >> 8) >= 15u) atomicSub(meta + b[u], 1u << 8);
  }
}


// The commit kernel, kCommitLanes lanes per plan, in two phases per plan: decide
// (header, claim check; for a loser its retry count) and apply (the writes).
// Between them each wavefront lists its losers for the next round: the
// atomic that reserves their list entries is issued before the writes and
// its result is used after them, so its latency hides behind them.
// Moves each commit lane fetches before it checks them (kCommitAhead) or
// writes them (kCommitAheadApply).  Four checks in flight took the mixed
// steady state (chains of 23 kicks on average at 97%) from 104 to 115 M
// ops/s; prefetching writes too cost the plain kernel a wavefront per SIMD,
// which the first rounds' one-move plans pay for.
constexpr int kCommitAhead = 4;
constexpr int kCommitAheadApply = 1;
constexpr uint32_t kMvSkip = 0x100;  // beyond the 8 flag bits: no move here
template <bool EXT>
__global__ __launch_bounds__(256) void k_commit(Geo g, Round r) {
  constexpr int CL = kCommitLanes;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (CL - 1);
  const int gshift = lane & ~(CL - 1);
  const bool leader = gl == 0;
  Pending P;
  P.init(r);
  // set by an earlier kernel: a plain load, once per wavefront, broadcast
  uint32_t ov = 0;
  if (lane == 0) ov = r.ctr->overflow;
  const bool void_round = __shfl(ov, 0, 64) != 0;
  const uint32_t passes = (P.n + kCommitOps - 1) / kCommitOps;
  for (uint32_t c = blockIdx.x; c < passes; c += gridDim.x) {
    const uint32_t pos = c * kCommitOps + threadIdx.x / CL;
    const uint32_t i = P.at(pos);
    // ---- decide ----
    uint32_t status = 0, twins = 0, nmv = 0, views = 0, off = 0, mv0_sf = 0, kicks = 0;
    uint32_t n_spawn = 0, spawn_off = 0, lost = 0, retries = 0, se = kNone;
    uint64_t x = 0, xa = 0;
    bool live = false, inl = true, win = false, requeue = false, abort = false;
    // move j of the plan: bin, slot, flags and the record it writes
    auto get = [&](uint32_t j, uint32_t& bin, uint32_t& slot, uint32_t& fl, uint64_t& k,
                   uint64_t& a) {
      if (inl) {
        uint32_t mb = off, msf = mv0_sf;
        if (j > 0) {
          const IMove m = r.imv[(size_t)i * kExtraInline + (j - 1)];
          mb = m.bin;
          msf = m.sf;
        }
        bin = mb;
        slot = msf & 0xFF;
        fl = msf >> 8;
        k = x;
        a = xa;
      } else {
        const Move m = r.arena[off + j];
        bin = m.bin;
        slot = m.slot;
        fl = m.flags;
        k = m.key;
        a = m.aux;
      }
    };
    if (i != kNone) {
      if (pos == 0 && leader && !void_round) atomicAdd(&r.ctr->rounds, 1u);
      if (void_round) {  // a planner ran out of arena: nothing of this round applies
        requeue = true;
      } else {
        live = true;
        // the header; the spawn record only for arena plans
        const uint4 h0 = r.hdr[i];
        status = h0.x & 0xF;
        twins = (h0.x >> 4) & 0xF;
        nmv = (h0.x >> 8) & 0xFFFFF;
        inl = (h0.x & kHdrArena) == 0;
        views = h0.y;
        off = h0.z;  // inline: the first move's bin; arena: the moves' offset
        mv0_sf = h0.w;
        se = (EXT && (h0.x & kHdrStash)) ? h0.w : kNone;  // the stash entry the plan writes
        kicks = (inl || se != kNone) ? 0u : h0.w;
        if (!inl) {
          const uint2 h1 = r.hdr_spawn[i];
          n_spawn = h1.x;
          spawn_off = h1.y;
        }
        x = r.keys[i];
        xa = ((inl || se != kNone) && r.vals) ? load_aux(r.vals, i, g.B) : 0;
        const unsigned long long me = r.tag | (unsigned long long)i;
        // kCommitAhead moves per lane in flight: a long chain's claim checks
        // are not one dependent load after another
        bool mine = true;
        for (uint32_t j0 = gl; j0 < nmv; j0 += CL * kCommitAhead) {
          uint32_t bn[kCommitAhead];
#pragma unroll
          for (int u = 0; u < kCommitAhead; ++u) {
            const uint32_t j = j0 + (uint32_t)u * CL;
            bn[u] = kNone;
            if (j < nmv) {
              uint32_t slot, fl;
              uint64_t k, a;
              get(j, bn[u], slot, fl, k, a);
            }
          }
#pragma unroll
          for (int u = 0; u < kCommitAhead; ++u)
            if (bn[u] != kNone && g.owner[bn[u]] != me) mine = false;
        }
        if (EXT && (h0.x & kHdrKeyClaim) && leader) {  // an upsert's claim on its key's first bin
          uint32_t kb[1];
          hash_key<1, EXT>(g, tab_of(g, r.op_table, r.tdesc, i), x, kb);
          if (g.owner[kb[0]] != me) mine = false;
        }
        if (EXT && se != kNone && leader && g.stash_owner[se] != me) mine = false;
        win = ((__ballot(!mine) >> gshift) & ((1ull << CL) - 1)) == 0;
        if (!win && leader) {
          lost = r.op_lost[i] + views;
          retries = r.op_retries[i] + 1;
          abort = r.max_rounds && retries >= r.max_rounds;
          requeue = !abort;
        }
      }
    }
    // ---- the ops that go again: segment u % kStripes of the next list
    // (u = this wavefront's index), one atomic add per wavefront that has any
    const bool rq = requeue && leader;
    const uint64_t bal = __ballot(rq);
    const uint32_t nrq = (uint32_t)__popcll(bal);
    const uint32_t sg = (c * 4 + (threadIdx.x >> 6)) % kStripes;
    uint32_t base = 0;
    if (nrq && lane == 0) base = atomicAdd(&r.next_cnt[sg * kStripeWords], nrq);
    // ---- apply ----
    if (live) {
      if (win) {
        // chain written from its end backwards (Sec. 8.2 system-transaction
        // order); each lane fetches its next kCommitAheadApply moves, then writes
        // them in the same order
        for (int top = (int)nmv - 1; top >= 0; top -= CL * kCommitAheadApply) {
          uint32_t bin[kCommitAheadApply], slot[kCommitAheadApply], fl[kCommitAheadApply];
          uint64_t k[kCommitAheadApply], a[kCommitAheadApply];
#pragma unroll
          for (int u = 0; u < kCommitAheadApply; ++u) {
            const int j = top - u * CL - gl;
            fl[u] = kMvSkip;
            if (j >= 0) get((uint32_t)j, bin[u], slot[u], fl[u], k[u], a[u]);
          }
#pragma unroll
          for (int u = 0; u < kCommitAheadApply; ++u) {
            if (fl[u] & kMvSkip) continue;
            uint32_t* mw = g.meta + bin[u];
            if (fl[u] & MV_DUPCLR) {
              atomicAnd(mw, ~(1u << slot[u]));
              continue;
            }
            if (fl[u] & MV_VALUE) {  // overwrite: the value word only
              unsigned long long* vw = &g.slots[(uint64_t)bin[u] * g.B + slot[u]].y;
              if (g.B == 1) *(uint32_t*)vw = (uint32_t)a[u];  // the rattle counter above stays
              else *vw = a[u];
            } else if (!(fl[u] & MV_SUPERSEDED)) {
              g.slots[(uint64_t)bin[u] * g.B + slot[u]] =
                  (fl[u] & MV_CLEAR) ? make_ulonglong2(kEmpty, 0ull) : make_ulonglong2(k[u], a[u]);
              if (g.ghost) {
                if (fl[u] & MV_DUP) atomicOr(mw, 1u << slot[u]);
                else atomicAnd(mw, ~(1u << slot[u]));
              }
            }
            if (fl[u] & MV_HC) atomicAdd(mw, 1u << 24);
          }
        }
        if (EXT && se != kNone && leader) {  // the stash entry: cleared, a new value, or the key
          ulonglong2* e = g.stash + se;
          uint32_t* cnt = g.stash_cnt + se / g.stash_n;
          if (r.is_delete && !r.overwrite) {
            *e = make_ulonglong2(kEmpty, 0ull);
            atomicSub(cnt, 1u);
          } else if (r.is_delete || status == PL_UPDATED) {
            e->y = xa;
          } else {
            *e = make_ulonglong2(x, xa);
            atomicAdd(cnt, 1u);
          }
        }
        if (leader) {
          uint8_t st;
          if (x == kEmpty) st = CK_OP_BAD_KEY;
          else if (r.is_delete) st = status == PL_OK ? CK_OP_OK : CK_OP_NOT_FOUND;
          else if (status == PL_OK) st = CK_OP_OK;
          else if (status == PL_UPDATED) st = CK_OP_UPDATED;
          else st = status == PL_STASHED ? CK_OP_STASHED : CK_OP_FAIL_CHAIN;
          r.status[i] = st;
          r.op_views[i] = views;
          if (kicks) r.op_kicks[i] = kicks;
          if (twins) r.op_twins[i] = twins;
        }
      } else if (leader) {
        r.op_lost[i] = lost;
        r.op_retries[i] = retries;
        if (abort) {
          r.status[i] = CK_OP_ABORTED;
          r.op_views[i] = 0;
        }
      }
      // spawn counts (Sec. 5) of every plan, committed or not, saturating at 15
      if (n_spawn) sc_increments(g.meta, r.spawns + spawn_off, n_spawn, (uint32_t)gl, CL);
    }
    if (nrq) {
      base = __shfl(base, 0, 64);
      if (rq) r.next[(size_t)sg * r.stripe_cap + base + __popcll(bal & ((1ull << lane) - 1))] = i;
    }
  }
}

hipError_t launch_commit(const Geo& g, const Round& r, hipStream_t s) {
  if (r.npend == 0) return hipSuccess;
  uint32_t grid = (uint32_t)(((uint64_t)r.npend + kCommitOps - 1) / kCommitOps);
  if (!r.first) grid = std::min(grid, kTailCommitBlocks);
  if (extended(g, r)) hipLaunchKernelGGL(k_commit<true>, dim3(grid), dim3(256), 0, s, g, r);
  else hipLaunchKernelGGL(k_commit<false>, dim3(grid), dim3(256), 0, s, g, r);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-sub-batch statistics
// ---------------------------------------------------------------------------
constexpr int kStatBlock = 256;

// The sub-batch still has pending ops (its last list is not empty), or the
// one before it has (its gate flag is set): the statistics kernels then leave
// everything untouched.  One wavefront per workgroup reads the counts; every
// thread of the workgroup calls it.  With `record`, workgroup 0 stores the
// outcome in `unfinished` (the next sub-batch's gate) and, when given, the
// host's summary of the sub-batch in pinned memory.
__device__ __forceinline__ bool stats_closed_out(const uint32_t* open, const uint32_t* gate,
                                                 uint32_t* unfinished, bool record,
                                                 const Ctr* c = nullptr,
                                                 HostSum* hsum = nullptr) {
  __shared__ uint32_t s_open;
  if (threadIdx.x < 64) {
    const bool own = open && list_open(open);  // all 64 lanes
    const bool o = (gate && *gate) || own;
    if (threadIdx.x == 0) {
      s_open = o ? 1u : 0u;
      if (record && blockIdx.x == 0) {
        *unfinished = o ? 1u : 0u;
        if (hsum) {  // for the host, straight to pinned memory
          hsum->done = own ? 0u : 1u;
          hsum->overflow = c->overflow;
          hsum->overflow_seen = c->overflow_seen;
          hsum->rounds = c->rounds;
        }
      }
    }
  }
  __syncthreads();
  return s_open != 0;
}

// Two passes over the sub-batch, both over the same partition: workgroup k
// takes tiles [k per, (k + 1) per) of kStatBlock ops (at most kStatMaxGrid
// workgroups, so the few same-address adds per workgroup stay cheap).  Blocks
// of 256 threads and at most 512 of them: 1024-thread blocks (at most 256)
// took 10.6 against 9.4 ms of statistics per benchmark step, and 2048
// workgroups 13.4.
struct StatSplit {
  uint32_t ntiles, per;
  __host__ __device__ StatSplit(uint64_t m, uint32_t grid)
      : ntiles((uint32_t)((m + kStatBlock - 1) / kStatBlock)),
        per((ntiles + grid - 1) / grid) {}
};
constexpr uint32_t kStatMaxGrid = 512;

// pass 1: successful inserts per workgroup; workgroup 0 snapshots `stored`
// (no other kernel of the sub-batch changes it before pass 2 has read it)
__global__ __launch_bounds__(kStatBlock) void k_stats_count(const uint8_t* status, uint64_t m,
                                                            uint32_t* block_ok,
                                                            uint64_t* stored_before,
                                                            const DevStats* st,
                                                            const uint32_t* open,
                                                            const uint32_t* gate,
                                                            uint32_t* unfinished, const Ctr* ctr,
                                                            HostSum* hsum) {
  __shared__ uint32_t s_w[kStatBlock / 64];
  const StatSplit sp(m, gridDim.x);
  const uint32_t t0 = blockIdx.x * sp.per, t1 = min(sp.ntiles, t0 + sp.per);
  // the status bytes are read before the gate check (unused if it is closed)
  uint32_t n = 0;
  for (uint32_t tile = t0; tile < t1; ++tile) {
    const uint64_t i = (uint64_t)tile * kStatBlock + threadIdx.x;
    // every key the sub-batch adds to the table, placed or stashed
    n += (i < m && (status[i] == CK_OP_OK || status[i] == CK_OP_STASHED)) ? 1u : 0u;
  }
  if (stats_closed_out(open, gate, unfinished, true, ctr, hsum)) return;
  n = (uint32_t)wave_sum(n);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kStatBlock / 64; ++w) tot += s_w[w];
    block_ok[blockIdx.x] = tot;
    if (blockIdx.x == 0) {
      unsigned long long stored = 0;
      for (int k = 0; k < kStatStripes; ++k) stored += st->s[k].v[S_STORED];
      *stored_before = stored;
    }
  }
}

// pass 2: the density band of every op and the totals.  An op's band comes
// from the number of successful inserts before it (its rank) on top of
// `stored` before the sub-batch; a tile whose first and last ranks fall in
// one band (nearly all: a band holds slots / CK_BANDS inserts) needs no
// per-op division.
__global__ __launch_bounds__(kStatBlock) void k_stats_apply(
    const uint8_t* status, const uint32_t* views, const uint32_t* lost, const uint32_t* kicks,
    const uint32_t* retries, const uint32_t* twins, uint64_t m, const uint32_t* block_ok,
    const uint64_t* stored_before, uint64_t slots, DevStats* st, const uint32_t* open,
    const uint32_t* gate) {
  const StatSplit sp(m, gridDim.x);
  const uint32_t t0 = blockIdx.x * sp.per, t1 = min(sp.ntiles, t0 + sp.per);
  // the per-op words of up to kAhead tiles, fetched together; the first
  // fetch is issued before the gate check and the prefix sum, whose
  // latencies it then overlaps (if the gate is closed the words go unused)
  constexpr int kAhead = 4;
  uint8_t sv[kAhead];
  uint32_t o_ret[kAhead], o_views[kAhead], o_lost[kAhead], o_kicks[kAhead], o_twins[kAhead];
  auto fetch = [&](uint32_t tb) {
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      const uint64_t idx = (uint64_t)(tb + q) * kStatBlock + threadIdx.x;
      const bool v = tb + q < t1 && idx < m;
      const uint64_t i = v ? idx : 0;  // every load in bounds, none behind a branch
      sv[q] = status[i];
      o_ret[q] = retries[i];
      o_views[q] = views[i];
      o_lost[q] = lost[i];
      o_kicks[q] = kicks[i];
      o_twins[q] = twins[i];
      // an upsert that gave a stored key its new value is not an insert
      if (!v || sv[q] == CK_OP_UPDATED) sv[q] = 0xFF;
    }
  };
  if (t0 < t1) fetch(t0);
  if (stats_closed_out(open, gate, nullptr, false)) return;
  __shared__ unsigned long long hb[4][CK_BANDS];
  __shared__ unsigned long long tot[12];
  __shared__ uint32_t wsum[kStatBlock / 64];
  __shared__ uint64_t s_rank0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < 4 * CK_BANDS; j += kStatBlock) hb[j / CK_BANDS][j % CK_BANDS] = 0;
  if (threadIdx.x < 12) tot[threadIdx.x] = 0;
  // successful inserts of the earlier workgroups (one wavefront sums them)
  if (wv == 0) {
    unsigned long long pre = 0;
    for (uint32_t k = lane; k < blockIdx.x; k += 64) pre += block_ok[k];
    pre = wave_sum(pre);
    if (lane == 0) s_rank0 = *stored_before + pre;
  }
  __syncthreads();
  unsigned long long a_ok = 0, a_fail = 0, a_abort = 0, a_bad = 0, a_views = 0, a_vall = 0,
                     a_kicks = 0, a_maxk = 0, a_ret = 0, a_tw = 0, a_stash = 0;
  // per-lane sums of the current band, added to the workgroup histogram when
  // the band changes and at the end
  uint32_t cb = kNone;
  unsigned long long c_n = 0, c_views = 0, c_kicks = 0, c_fail = 0;
  auto flush = [&]() {
    if (cb != kNone) {
      if (c_n) atomicAdd(&hb[0][cb], c_n);
      if (c_views) atomicAdd(&hb[1][cb], c_views);
      if (c_kicks) atomicAdd(&hb[2][cb], c_kicks);
      if (c_fail) atomicAdd(&hb[3][cb], c_fail);
    }
    c_n = c_views = c_kicks = c_fail = 0;
  };
  auto band_of = [&](uint64_t stored) -> uint32_t {
    const uint64_t b = (uint64_t)CK_BANDS * stored / slots;
    return (uint32_t)(b >= CK_BANDS ? CK_BANDS - 1 : b);
  };
  uint64_t rank0 = s_rank0;
  // the band at the workgroup's first rank and the first rank of the next
  // band: below it an op's band needs no division (bands hold slots /
  // CK_BANDS inserts, so a workgroup's ranks rarely cross one)
  uint32_t cb0 = 0;
  uint64_t next_edge = ~0ull;
  if (slots) {
    cb0 = band_of(rank0);
    if (cb0 + 1 < CK_BANDS) next_edge = ((uint64_t)(cb0 + 1) * slots + CK_BANDS - 1) / CK_BANDS;
  }
  for (uint32_t tb = t0; tb < t1; tb += kAhead) {
    if (tb != t0) fetch(tb);
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      if (tb + q >= t1) break;  // uniform
      const uint8_t s = sv[q];
      const bool ok = s == CK_OP_OK;
      // the rank counts every key held: placed or stashed
      const uint64_t bal = __ballot(ok || s == CK_OP_STASHED);
      const uint32_t before_in_wave = __popcll(bal & ((1ull << lane) - 1));
      if (lane == 0) wsum[wv] = __popcll(bal);
      __syncthreads();
      uint32_t wpre = 0, ttot = 0;
      for (int w = 0; w < kStatBlock / 64; ++w) {
        const uint32_t c = wsum[w];
        wpre += w < wv ? c : 0u;
        ttot += c;
      }
      __syncthreads();  // wsum is rewritten by the next tile
      const uint64_t rank = rank0 + wpre + before_in_wave;
      uint32_t band = 0;
      bool banded = false;
      if (s != 0xFF) {
        if (s == CK_OP_BAD_KEY) {
          a_bad += 1;
        } else {
          a_ret += o_ret[q];
          a_vall += (unsigned long long)o_views[q] + o_lost[q];
          if (s == CK_OP_ABORTED) {
            a_abort += 1;
          } else {
            if (slots) {  // a group of tables has no single density: totals only
              band = rank < next_edge ? cb0 : band_of(rank);
              banded = true;
            }
            a_views += o_views[q];
            if (ok) {
              a_ok += 1;
              a_kicks += o_kicks[q];
              a_maxk = o_kicks[q] > a_maxk ? o_kicks[q] : a_maxk;
              a_tw += o_twins[q];
            } else if (s == CK_OP_STASHED) {  // a failed chain all the same
              a_stash += 1;
            } else {
              a_fail += 1;
            }
          }
        }
      }
      if (banded) {
        if (band != cb) {
          flush();
          cb = band;
        }
        c_n += 1;
        c_views += o_views[q];
        if (ok) c_kicks += o_kicks[q];
        else c_fail += 1;
      }
      rank0 += ttot;
    }
  }
  flush();
  a_ok = wave_sum(a_ok); a_fail = wave_sum(a_fail); a_abort = wave_sum(a_abort);
  a_bad = wave_sum(a_bad); a_views = wave_sum(a_views); a_vall = wave_sum(a_vall);
  a_kicks = wave_sum(a_kicks); a_maxk = wave_max(a_maxk); a_ret = wave_sum(a_ret);
  a_tw = wave_sum(a_tw); a_stash = wave_sum(a_stash);
  if (lane == 0) {
    atomicAdd(&tot[0], a_ok); atomicAdd(&tot[1], a_fail); atomicAdd(&tot[2], a_abort);
    atomicAdd(&tot[3], a_bad); atomicAdd(&tot[4], a_views); atomicAdd(&tot[5], a_vall);
    atomicAdd(&tot[6], a_kicks); atomicMax(&tot[7], a_maxk); atomicAdd(&tot[8], a_ret);
    atomicAdd(&tot[9], a_tw); atomicAdd(&tot[10], a_stash);
  }
  __syncthreads();
  DevStatLine& sl = st->s[blockIdx.x % kStatStripes];
  if (threadIdx.x < 11) {
    const int map[11] = {S_INS_OK, S_INS_FAIL, S_INS_ABORT, S_INS_BAD, S_VIEWS,
                         S_VIEWS_ALL, S_KICKS, S_MAX_KICKS, S_RETRIES, S_TWINS,
                         S_INS_STASHED};
    const int j = threadIdx.x;
    if (tot[j]) {
      if (j == 7) atomicMax(&sl.v[S_MAX_KICKS], tot[j]);
      else atomicAdd(&sl.v[map[j]], tot[j]);
    }
    // `stored` grows by this workgroup's successful inserts, placed or stashed
    if (j == 0 && tot[0] + tot[10]) atomicAdd(&sl.v[S_STORED], tot[0] + tot[10]);
  }
  for (int j = threadIdx.x; j < 4 * CK_BANDS; j += kStatBlock) {
    const unsigned long long v = hb[j / CK_BANDS][j % CK_BANDS];
    if (v) atomicAdd(&sl.band[j / CK_BANDS][j % CK_BANDS], v);
  }
}

// deletes: found/probes/retries totals; `stored` decreases by the found count
__global__ __launch_bounds__(kStatBlock) void k_stats_delete(const uint8_t* status,
                                                             const uint32_t* probes,
                                                             const uint32_t* retries, uint64_t m,
                                                             DevStats* st, const uint32_t* open,
                                                             const uint32_t* gate,
                                                             uint32_t* unfinished,
                                                             uint32_t count, const Ctr* ctr,
                                                             HostSum* hsum) {
  if (stats_closed_out(open, gate, unfinished, true, ctr, hsum)) return;
  if (!count) return;  // overwrites: no counters, only the completion flag
  unsigned long long d = 0, f = 0, p = 0, rt = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (status[i] != CK_OP_BAD_KEY) {
      d += 1;
      f += status[i] == CK_OP_OK;
      p += probes[i];
      rt += retries[i];
    }
  }
  d = wave_sum(d); f = wave_sum(f); p = wave_sum(p); rt = wave_sum(rt);
  if ((threadIdx.x & 63) == 0) {
    DevStatLine& sl = st->s[(blockIdx.x * (kStatBlock / 64) + (threadIdx.x >> 6)) % kStatStripes];
    if (d) atomicAdd(&sl.v[S_DELETES], d);
    if (f) {
      atomicAdd(&sl.v[S_DEL_FOUND], f);
      atomicAdd(&sl.v[S_STORED], (unsigned long long)(0ull - f));
    }
    if (p) atomicAdd(&sl.v[S_DEL_PROBES], p);
    if (rt) atomicAdd(&sl.v[S_DEL_RETRIES], rt);
  }
}

size_t stats_tmp_words(uint64_t m) {
  const uint64_t nb = (m + kStatBlock - 1) / kStatBlock;
  return ((nb + 63) & ~(uint64_t)63) + 16;  // per-workgroup counts, then `stored` before
}

hipError_t launch_batch_stats(const Round& r, uint64_t m, uint64_t slots, uint32_t* block_tmp,
                              uint32_t is_delete, const uint32_t* open, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)((m + kStatBlock - 1) / kStatBlock);
  if (is_delete) {
    hipLaunchKernelGGL(k_stats_delete, dim3(std::min<uint32_t>(nb, kStatMaxGrid)), dim3(kStatBlock), 0, s,
                       r.status, r.op_views, r.op_retries, m, r.stats, open, r.gate,
                       &r.ctr->unfinished, r.overwrite ? 0u : 1u, r.ctr, r.hsum);
    return hipGetLastError();
  }
  uint64_t* stored_before = (uint64_t*)(block_tmp + ((nb + 63) & ~63u));
  const uint32_t grid = std::min<uint32_t>(nb, kStatMaxGrid);
  hipLaunchKernelGGL(k_stats_count, dim3(grid), dim3(kStatBlock), 0, s, r.status, m, block_tmp,
                     stored_before, r.stats, open, r.gate, &r.ctr->unfinished, r.ctr, r.hsum);
  hipLaunchKernelGGL(k_stats_apply, dim3(grid), dim3(kStatBlock), 0, s, r.status, r.op_views,
                     r.op_lost, r.op_kicks, r.op_retries, r.op_twins, m, block_tmp,
                     stored_before, slots, r.stats, open, r.gate);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// transactional batches (Sec. 8): one lane per transaction
// ---------------------------------------------------------------------------
// A lane plans its transaction's operations in order against the round-start
// table through a private overlay in scratch: every bin the plan has touched
// (read or written), each a copy of the bin's slots and metadata word, so
// that later operations see the earlier ones' writes.  The overlay is the
// transaction's read set and write set at once: every bin in it is claimed
// with the transaction's index (the smallest index wins a bin), and a
// transaction that owns all of them commits by writing back the bins it
// changed; the others plan again next round.  An insert runs the table's
// walk (random kicking, or queue-kicking with its hit counters) inside the
// overlay, kick-out chain included; a failed insert is undone from a log of
// the slots and words it overwrote (the bins it read stay in the overlay,
// and so in the read set).  A plan that would touch more than kTxnBins bins
// aborts.

template <int B>
struct TxnLane {
  const Geo* g;
  uint32_t* bins;    // [kTxnBins]
  uint32_t* meta;    // [kTxnBins]
  uint32_t* dirty;   // [kTxnBins]: 1 once written
  ulonglong2* slots; // [kTxnBins * B]
  uint32_t* uent;    // undo log of the current insert: entry, slot,
  uint32_t* uslot;   // previous slot contents and word
  ulonglong2* uold;
  uint32_t* umeta;
  uint32_t n = 0, nu = 0;
  bool big = false;

  __device__ void init(const Geo& geo, char* base, uint32_t undo_cap) {
    g = &geo;
    bins = (uint32_t*)base;
    meta = bins + kTxnBins;
    dirty = meta + kTxnBins;
    slots = (ulonglong2*)(dirty + kTxnBins);
    uent = (uint32_t*)(slots + (size_t)kTxnBins * B);
    uslot = uent + undo_cap;
    umeta = uslot + undo_cap;
    uold = (ulonglong2*)(umeta + undo_cap);  // undo_cap is a multiple of 4: 16-byte aligned
  }
  // Overlay entry of bin b, copied from the table on first touch; kNone
  // (and big) when the overlay is full.
  __device__ uint32_t touch(uint32_t b) {
    for (uint32_t e = 0; e < n; ++e)
      if (bins[e] == b) return e;
    if (n == kTxnBins) {
      big = true;
      return kNone;
    }
    bins[n] = b;
    meta[n] = g->meta[b];
    dirty[n] = 0;
#pragma unroll
    for (int s = 0; s < B; ++s) slots[(size_t)n * B + s] = g->slots[(uint64_t)b * B + s];
    return n++;
  }
  __device__ int first_empty(uint32_t e) const {
#pragma unroll
    for (int s = 0; s < B; ++s)
      if (slots[(size_t)e * B + s].x == kEmpty) return s;
    return -1;
  }
  __device__ int occupancy(uint32_t e) const {
    int o = 0;
#pragma unroll
    for (int s = 0; s < B; ++s) o += slots[(size_t)e * B + s].x != kEmpty;
    return o;
  }
  // slot s of entry e gets rec (an insertion: queue-kicking counts it)
  __device__ void put(uint32_t e, int s, ulonglong2 rec, bool log) {
    ulonglong2& sl = slots[(size_t)e * B + s];
    if (log) {
      uent[nu] = e;
      uslot[nu] = (uint32_t)s;
      uold[nu] = sl;
      umeta[nu] = meta[e];
      ++nu;
    }
    sl = rec;
    dirty[e] = 1;
    if (g->scheme == CK_QUEUE) meta[e] += 1u << 24;
  }
  __device__ void undo() {
    while (nu) {
      --nu;
      slots[(size_t)uent[nu] * B + uslot[nu]] = uold[nu];
      meta[uent[nu]] = umeta[nu];
    }
  }
  // the entry and slot holding key x among its bins (h in hash order)
  __device__ bool find(uint64_t x, const uint32_t* h, uint32_t& e, int& s) {
    for (int i = 0; i < 2; ++i) {
      e = touch(h[i]);
      if (big) return false;
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (slots[(size_t)e * B + q].x == x) {
          s = q;
          return true;
        }
    }
    return false;
  }
  // Insert x (absent) by the table's walk; PL_OK or PL_FAIL (a failed
  // insert leaves the overlay's contents as they were).
  __device__ uint32_t insert(ulonglong2 x, uint64_t op, const uint32_t* h) {
    nu = 0;
    uint32_t draws = 0, kicks = 0;
    const bool queue = g->scheme == CK_QUEUE;
    uint32_t e0 = kNone, e1 = kNone;
    if (g->balance || queue) {  // load balancing (Sec. 2; always for queue-kicking)
      e0 = touch(h[0]);
      if (big) return PL_FAIL;
      e1 = touch(h[1]);
      if (big) return PL_FAIL;
      const int o0 = occupancy(e0), o1 = occupancy(e1);
      if (o0 < B || o1 < B) {
        const uint32_t t = o0 <= o1 ? e0 : e1;
        put(t, first_empty(t), x, false);
        return PL_OK;
      }
    } else {  // first fit (Sec. 1)
      e0 = touch(h[0]);
      if (big) return PL_FAIL;
      int fe = first_empty(e0);
      if (fe >= 0) {
        put(e0, fe, x, false);
        return PL_OK;
      }
      e1 = touch(h[1]);
      if (big) return PL_FAIL;
      fe = first_empty(e1);
      if (fe >= 0) {
        put(e1, fe, x, false);
        return PL_OK;
      }
    }
    // kick-out walk: hit balancing picks the bin (queue), else a random one
    uint32_t cur;
    if (queue) cur = (meta[e0] >> 24) <= (meta[e1] >> 24) ? e0 : e1;
    else cur = uniform_choice(*g, op, draws, 2) == 0 ? e0 : e1;
    ulonglong2 carry = x;
    for (;;) {
      if (kicks == g->max_chain) {
        undo();
        return PL_FAIL;
      }
      const int s = queue ? (int)((meta[cur] >> 24) % B) : (int)uniform_choice(*g, op, draws, B);
      const ulonglong2 victim = slots[(size_t)cur * B + s];
      put(cur, s, carry, true);
      ++kicks;
      carry = victim;
      uint32_t hv[2];
      hash_key<2, false>(*g, Tab{0u, g->n}, carry.x, hv);
      const uint32_t nb = hv[0] == bins[cur] ? hv[1] : hv[0];
      cur = touch(nb);
      if (big) {
        undo();
        return PL_FAIL;
      }
      const int fe = first_empty(cur);
      if (fe >= 0) {
        put(cur, fe, carry, true);
        return PL_OK;
      }
    }
  }
};

template <int B>
__global__ __launch_bounds__(256) void k_plan_txn(Geo g, TxnRound r) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.npend) return;
  const uint32_t i = r.pend ? r.pend[p] : p;  // the transaction, within the sub-batch
  const uint32_t t = r.t0 + i;
  TxnLane<B> L;
  L.init(g, r.scratch + (size_t)p * r.lane_bytes, r.undo_cap);
  const uint32_t o0 = r.off[t], o1 = r.off[t + 1];
  for (uint32_t j = o0; j < o1 && !L.big; ++j) {
    const uint64_t x = r.keys[j];
    uint8_t st = CK_OP_NOT_FOUND;
    uint64_t v = 0;
    if (x == kEmpty) {
      st = CK_OP_BAD_KEY;
    } else {
      uint32_t h[2];
      hash_key<2, false>(g, Tab{0u, g.n}, x, h);
      const uint32_t kd = r.kind[j];
      uint32_t e = 0;
      int s = 0;
      if (kd == TXN_INSERT) {
        st = L.insert(make_ulonglong2(x, r.vals[j]), r.op_base + j, h) == PL_OK ? CK_OP_OK
                                                                             : CK_OP_FAIL_CHAIN;
      } else if (L.find(x, h, e, s)) {
        st = CK_OP_OK;
        ulonglong2& sl = L.slots[(size_t)e * B + s];
        if (kd == TXN_LOOKUP) {
          v = sl.y;
        } else if (kd == TXN_DELETE) {
          sl = make_ulonglong2(kEmpty, 0ull);
          L.dirty[e] = 1;
        } else {  // overwrite
          sl.y = r.vals[j];
          L.dirty[e] = 1;
        }
      }
    }
    r.status[j] = st;
    r.vout[j] = v;
  }
  if (L.big) {  // too many bins: the transaction aborts, claiming nothing
    r.nob[p] = kNone;
    return;
  }
  r.nob[p] = L.n;
  const unsigned long long me = r.tag | (unsigned long long)i;
  for (uint32_t e = 0; e < L.n; ++e) atomicMin(&g.owner[L.bins[e]], me);
}

template <int B>
__global__ __launch_bounds__(256) void k_commit_txn(Geo g, TxnRound r) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= r.npend) return;
  const uint32_t i = r.pend ? r.pend[p] : p;
  const uint32_t t = r.t0 + i;
  const uint32_t o0 = r.off[t], o1 = r.off[t + 1];
  const uint32_t n = r.nob[p];
  TxnLane<B> L;
  L.init(g, r.scratch + (size_t)p * r.lane_bytes, r.undo_cap);
  bool win = n != kNone;
  const unsigned long long me = r.tag | (unsigned long long)i;
  for (uint32_t e = 0; win && e < n; ++e) win = g.owner[L.bins[e]] == me;
  bool abort = n == kNone;
  if (!win && !abort) {
    const uint32_t lost = ++r.lost[i];
    abort = r.max_rounds && lost >= r.max_rounds;
  }
  if (win) {
    for (uint32_t e = 0; e < n; ++e) {
      if (!L.dirty[e]) continue;
      const uint32_t b = L.bins[e];
#pragma unroll
      for (int s = 0; s < B; ++s) g.slots[(uint64_t)b * B + s] = L.slots[(size_t)e * B + s];
      g.meta[b] = L.meta[e];
    }
    unsigned long long ok = 0, fail = 0, del = 0;
    for (uint32_t j = o0; j < o1; ++j) {
      const uint8_t st = r.status[j];
      const uint32_t kd = r.kind[j];
      ok += kd == TXN_INSERT && st == CK_OP_OK;
      fail += kd == TXN_INSERT && st == CK_OP_FAIL_CHAIN;
      del += kd == TXN_DELETE && st == CK_OP_OK;
    }
    DevStatLine& sl = r.stats->s[blockIdx.x % kStatStripes];
    if (ok) atomicAdd(&sl.v[S_INS_OK], ok);
    if (fail) atomicAdd(&sl.v[S_INS_FAIL], fail);
    if (del) atomicAdd(&sl.v[S_DEL_FOUND], del);
    if (ok != del) atomicAdd(&sl.v[S_STORED], ok - del);
    r.txn_round[t] = r.round;
  } else if (abort) {
    for (uint32_t j = o0; j < o1; ++j) {
      r.status[j] = CK_OP_ABORTED;
      r.vout[j] = 0;
    }
    r.txn_round[t] = r.round;
  } else {
    const uint32_t q = atomicAdd(r.next_cnt, 1u);
    r.next[q] = i;
  }
}

// Undo-log records per lane: every kick of an insert's walk and its final
// placement, rounded up to a multiple of 4.
uint32_t txn_undo_cap(const Geo& g) { return (g.max_chain + 2 + 3) & ~3u; }

// Scratch bytes of one lane: bins, words and dirty flags (4 bytes each per
// entry), the entries' slots, and the undo log (entry, slot, word, old slot).
size_t txn_lane_bytes(const Geo& g) {
  const size_t uc = txn_undo_cap(g);
  const size_t b = (size_t)kTxnBins * 12 + (size_t)kTxnBins * g.B * 16 + uc * 12 + uc * 16;
  return (b + 255) & ~(size_t)255;
}

template <int B>
static void txn_go(const Geo& g, const TxnRound& r, bool commit, hipStream_t s) {
  const uint32_t grid = (r.npend + 255) / 256;
  if (commit) hipLaunchKernelGGL(k_commit_txn<B>, dim3(grid), dim3(256), 0, s, g, r);
  else hipLaunchKernelGGL(k_plan_txn<B>, dim3(grid), dim3(256), 0, s, g, r);
}

hipError_t launch_txn(const Geo& g, const TxnRound& r, bool commit, hipStream_t s) {
  if (r.npend == 0) return hipSuccess;
  switch (g.B) {
    case 2: txn_go<2>(g, r, commit, s); break;
    case 4: txn_go<4>(g, r, commit, s); break;
    case 8: txn_go<8>(g, r, commit, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ck
