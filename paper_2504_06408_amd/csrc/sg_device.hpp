// Device building blocks shared by the gfx950 kernels: wavefront-64 scans and
// reductions, a block-wide exclusive scan, the LDS open-addressing hash used
// to find an output slot for a column id, an LDS bitonic sort, and the
// flattened product iterator that spreads the uneven B-row segments of one
// output row evenly over a workgroup's lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SG_DEV __device__ __forceinline__

namespace sg {

constexpr int kWave = 64;
constexpr int32_t kEmptyKey = -1;

SG_DEV int lane_id() { return (int)__lane_id(); }

// Workgroup barrier for kernels whose wavefronts exchange data through LDS
// only: the fences cover LDS alone, so a wavefront waits for its own LDS
// operations (lgkmcnt) but not for its outstanding global loads and stores,
// which __syncthreads() would also drain.
SG_DEV void block_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
SG_DEV int wave_id() { return (int)(threadIdx.x >> 6); }

// Orders the LDS accesses of one wavefront whose lanes exchange data through
// LDS with no workgroup barrier: its LDS operations complete before any
// lane goes on.
SG_DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

SG_DEV unsigned long long lanes_below() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <class T>
SG_DEV T shfl(T v, int src) {
  return __shfl(v, src, kWave);
}

// x of the lane that the DPP control kCtrl selects (within the rows enabled
// by kRowMask); lanes with no source lane, or in a disabled row, get 0.
// 8-byte values move as two 32-bit halves from the same source lane.
template <int kCtrl, int kRowMask, bool kBoundZero, class T>
SG_DEV T dpp_from(T x) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte lane values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, kRowMask, 0xf, kBoundZero));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, kCtrl, kRowMask, 0xf, kBoundZero);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), kCtrl, kRowMask, 0xf, kBoundZero);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// Inclusive prefix sum over the 64 lanes of a wavefront, in registers: shifts
// by 1, 2, 4, 8 lanes inside each row of 16 (row_shr), then the last lane of
// row 0 and 2 is added to rows 1 and 3 (row_bcast:15) and the last lane of
// row 1 to rows 2 and 3 (row_bcast:31).  Every lane must be active.
template <class T>
SG_DEV T wave_incl_scan(T v) {
  v += dpp_from<0x111, 0xf, true>(v);
  v += dpp_from<0x112, 0xf, true>(v);
  v += dpp_from<0x114, 0xf, true>(v);
  v += dpp_from<0x118, 0xf, true>(v);
  v += dpp_from<0x142, 0xa, false>(v);
  v += dpp_from<0x143, 0xc, false>(v);
  return v;
}

// A block- or wavefront-uniform value read from the first active lane, so
// the compiler can keep it (and addresses built on it) in scalar registers.
SG_DEV int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The value that lane l holds, in every lane.
template <class T>
SG_DEV T lane_value(T x, int l) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte lane values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// Sum over the 64 lanes, in every lane.  Every lane must be active.
template <class T>
SG_DEV T wave_sum(T v) {
  return lane_value(wave_incl_scan(v), kWave - 1);
}

template <class T>
SG_DEV T wave_max(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    T u = __shfl_xor(v, d, kWave);
    v = u > v ? u : v;
  }
  return v;
}

// Block-wide exclusive scan for NW wavefronts.  s_wave: NW slots of LDS.
// Returns the exclusive prefix of v; *total receives the block sum.  Every
// thread of the block must call it (it contains barriers).
template <int NW, class T>
SG_DEV T block_excl_scan(T v, T* s_wave, T* total) {
  const T incl = wave_incl_scan(v);
  if (lane_id() == kWave - 1) s_wave[wave_id()] = incl;
  block_sync();
  T pre = 0, tot = 0;
  const int w = wave_id();
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const T s = s_wave[i];
    pre += (i < w) ? s : (T)0;
    tot += s;
  }
  *total = tot;
  block_sync();
  return pre + incl - v;
}

template <int NW, class T>
SG_DEV T block_sum(T v, T* s_wave) {
  T tot;
  (void)block_excl_scan<NW, T>(v, s_wave, &tot);
  return tot;
}

SG_DEV int ceil_log2_u64(uint64_t x) { return x <= 1 ? 0 : 64 - __clzll((long long)(x - 1)); }

// ---------------------------------------------------------------------------
// LDS hash of int32 column ids, linear probing, power-of-two size 2^lgS.
// Multiplicative hashing spreads the clustered low column ids of power-law
// graphs.  The table must never fill up (callers size it >= 2x keys).
SG_DEV uint32_t hash_home(int32_t key, int lgS) { return ((uint32_t)key * 0x9E3779B1u) >> (32 - lgS); }

// Find or claim the slot of `key`; *fresh tells whether this call claimed it.
// Returns kHashFull after probing every slot without success (a full table,
// which only inconsistent inputs can cause), so a wave never spins forever.
constexpr uint32_t kHashFull = 0xFFFFFFFFu;
SG_DEV uint32_t hash_insert(int32_t* keys, int lgS, int32_t key, bool* fresh) {
  const uint32_t mask = (1u << lgS) - 1u;
  uint32_t s = hash_home(key, lgS);
  *fresh = false;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    int32_t cur = __hip_atomic_load(keys + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == key) {
      *fresh = false;
      return s;
    }
    if (cur == kEmptyKey) {
      const int32_t old = atomicCAS(keys + s, kEmptyKey, key);
      if (old == kEmptyKey) {
        *fresh = true;
        return s;
      }
      if (old == key) {
        *fresh = false;
        return s;
      }
    }
    s = (s + 1u) & mask;
  }
  return kHashFull;
}

// ---------------------------------------------------------------------------
// Ascending bitonic sort of n (power of two) 64-bit keys in LDS by a whole
// workgroup of BS threads.  Contains barriers.
template <int BS>
SG_DEV void block_bitonic_sort(uint64_t* buf, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int x = threadIdx.x; x < (n >> 1); x += BS) {
        const int i = 2 * x - (x & (j - 1));
        const int l = i + j;
        const uint64_t a = buf[i], b = buf[l];
        const bool up = (i & k) == 0;
        if ((a > b) == up) {
          buf[i] = b;
          buf[l] = a;
        }
      }
      block_sync();
    }
  }
}

// Stable LSD radix sort of n (<= NMAX) 64-bit items in LDS by the key bits
// [32, 32 + kbits) (8-bit digits) by a workgroup of BS >= 256 threads.  Each
// wavefront owns a contiguous chunk of the items and ranks 64 of them per
// round: lanes with the same digit are found with eight ballots, and a
// per-(wave, digit) counter in LDS carries the running count, so equal digits
// keep their order.  A 256-digit scan then gives every (wave, digit) its
// output offset.  buf and tmp hold NMAX items each; s_hist has NW*256 ints,
// s_wt 4 ints.  Returns the buffer that holds the sorted items.
template <int BS, int NMAX>
SG_DEV uint64_t* block_radix_sort_hi(uint64_t* buf, uint64_t* tmp, int n, int kbits, int32_t* s_hist,
                                     int32_t* s_wt) {
  static_assert(BS >= 256, "one thread per digit");
  constexpr int NW = BS / kWave;
  constexpr int RPL = (NMAX + BS - 1) / BS;
  const int w = wave_id(), l = lane_id();
  const int per_wave = (n + NW - 1) / NW;
  const int c0 = w * per_wave;
  const int c1 = (c0 + per_wave) < n ? (c0 + per_wave) : n;
  for (int shift = 32; shift < 32 + kbits; shift += 8) {
    for (int x = threadIdx.x; x < NW * 256; x += BS) s_hist[x] = 0;
    block_sync();
    uint64_t item[RPL];
    int rank[RPL], dig[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int x = c0 + r * kWave + l;
      const bool valid = x < c1;
      const uint64_t v = valid ? buf[x] : 0ull;
      const int d = valid ? (int)((v >> shift) & 255u) : 0;
      unsigned long long m = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool on = (d >> b) & 1;
        const unsigned long long bb = __ballot(on);
        m &= on ? bb : ~bb;
      }
      const unsigned long long below = m & lanes_below();
      int32_t* slot = s_hist + w * 256 + d;
      const int old = valid ? *slot : 0;
      if (valid && below == 0) *slot = old + __popcll(m);
      item[r] = v;
      rank[r] = old + __popcll(below);
      dig[r] = valid ? d : -1;
    }
    block_sync();
    // waves 0..3 (threads 0..255) own one digit each
    int tot = 0, inc = 0;
    if (threadIdx.x < 256) {
      for (int q = 0; q < NW; ++q) tot += s_hist[q * 256 + threadIdx.x];
      inc = wave_incl_scan(tot);
      if (l == kWave - 1) s_wt[w] = inc;
    }
    block_sync();
    if (threadIdx.x < 256) {
      const int d = threadIdx.x;
      int run = inc - tot;
      for (int q = 0; q < w; ++q) run += s_wt[q];
      for (int q = 0; q < NW; ++q) {
        const int t = s_hist[q * 256 + d];
        s_hist[q * 256 + d] = run;
        run += t;
      }
    }
    block_sync();
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (dig[r] >= 0) tmp[s_hist[w * 256 + dig[r]] + rank[r]] = item[r];
    block_sync();
    uint64_t* t = buf;
    buf = tmp;
    tmp = t;
  }
  return buf;
}

// Ascending bitonic sort across the 64 lanes of a wavefront of (key, payload)
// pairs, keys compared as signed int32.
template <class P>
SG_DEV void wave_bitonic_sort(int32_t& key, P& pay) {
  const int l = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int32_t ok = __shfl_xor(key, j, kWave);
      const P op = __shfl_xor(pay, j, kWave);
      const bool lower = (l & j) == 0;
      const bool up = (l & k) == 0;
      // the lower lane of a pair keeps the smaller key when sorting up
      const bool take_other = (lower == up) ? (ok < key) : (ok > key);
      if (take_other) {
        key = ok;
        pay = op;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Flattened product iteration for one output row by a whole workgroup.
//
// An output row is fed by `nsrc` sources (A's stored entries of the row, or
// the parts of a merge); source j contributes a segment of `len` consecutive
// entries starting at `start` in its own arrays.  Lengths are very uneven
// (power-law B rows), so instead of one lane per source the sources are taken
// BS at a time, their lengths are prefix-summed, and product q of the chunk
// goes to lane q mod BS: lane loads of one segment are contiguous and every
// lane does the same amount of work.
//
// Src provides:
//   using Item;                              per-source payload kept in LDS
//   SG_DEV void load(int64_t j, Item& it, int64_t& start, int64_t& len) const;
// fetch(const Item&, int64_t idx) reads one product from global memory (idx
// is its index in the source's arrays) and returns it by value; apply(p)
// folds it into LDS.  Each lane first fetches U products (U independent loads
// in flight, so the gathers are not serialised behind the LDS updates) and
// then applies them.
// One chunk's sources [c0, c0 + BS) into compacted slots (see above);
// returns the chunk's product count, *nc its slots.
template <int BS, class Src>
SG_DEV int64_t product_chunk(const Src& src, int64_t nsrc, int64_t c0, typename Src::Item* s_item, int64_t* s_start,
                             int64_t* s_off, int64_t* s_wave, int* nc) {
  constexpr int NW = BS / kWave;
  const int64_t j = c0 + threadIdx.x;
  int64_t start = 0, len = 0;
  typename Src::Item it{};
  if (j < nsrc) src.load(j, it, start, len);
  // sources with an empty segment are dropped: one scan of (length, flag)
  // pairs gives each non-empty source its slot and first product; a slot
  // keeps its segment start minus that offset, so product q of slot k is
  // element s_start[k] + q of its source
  const int64_t pk = (len << 16) | (len > 0 ? 1 : 0);
  int64_t tot;
  const int64_t ex = block_excl_scan<NW, int64_t>(pk, s_wave, &tot);
  if (len > 0) {
    const int pos = (int)(ex & 0xffff);
    s_item[pos] = it;
    s_off[pos] = ex >> 16;
    s_start[pos] = start - (ex >> 16);
  }
  *nc = (int)(tot & 0xffff);
  block_sync();
  return tot >> 16;
}

// The products of block [qb, qb + 64*U) of a chunk of nc slots and `total`
// products: lane l fetches q = qb + u*64 + l into p[u] (ok[u]: q < total).
// The owners of the block's first and last product come from a 64-ary
// search (one LDS read per lane and level); each lane then searches only the
// slots in between, starting from its previous hit.  All searches come
// first, then all U fetches (their loads in flight together).
template <int BS, int U, class Src, class Fetch, class P>
SG_DEV void product_block(const typename Src::Item* s_item, const int64_t* s_start, const int64_t* s_off, int nc,
                          int64_t total, int64_t qb, Fetch& fetch, P* p, bool* ok) {
  constexpr int64_t kBlock = (int64_t)kWave * U;
  const int lane = lane_id();
  // odd, so that the lanes' 8-byte offset reads spread over all LDS banks
  const int stride = ((nc + kWave - 1) / kWave) | 1;
  const int64_t qe = (qb + kBlock - 1) < (total - 1) ? (qb + kBlock - 1) : (total - 1);
  int a, e;
  {
    const int i1 = lane * stride;
    const int64_t o1 = i1 < nc ? s_off[i1] : INT64_MAX;
    const int ca = __popcll(__ballot(o1 <= qb)), ce = __popcll(__ballot(o1 <= qe));
    const int ba = (ca - 1) * stride, be = (ce - 1) * stride;
    const int l2 = lane & 31;
    const int i2 = (lane < 32 ? ba : be) + l2;
    const int64_t o2 = (l2 < stride && i2 < nc) ? s_off[i2] : INT64_MAX;
    const unsigned long long m2 = __ballot(o2 <= (lane < 32 ? qb : qe));
    a = ba + __popc((uint32_t)m2) - 1;
    e = be + __popc((uint32_t)(m2 >> 32)) - 1;
  }
  int own[U];
  int lo = a;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t q = qb + u * kWave + lane;
    ok[u] = q < total;
    if (ok[u]) {
      int hi = e;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
    }
    own[u] = lo;
  }
  // lanes past the chunk's end fetch the block's first product, which
  // always exists
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = ok[u] ? own[u] : a;
    const int64_t q = ok[u] ? qb + u * kWave + lane : qb;
    p[u] = fetch(s_item[k], s_start[k] + q);
  }
}

template <int BS, int U, class Src, class Fetch, class Apply>
SG_DEV void for_each_product(const Src& src, int64_t nsrc, typename Src::Item* s_item, int64_t* s_start,
                             int64_t* s_off, int64_t* s_wave, Fetch& fetch, Apply& apply) {
  constexpr int NW = BS / kWave;
  static_assert(BS < (1 << 16) && (((BS + kWave - 1) / kWave) | 1) <= kWave / 2,
                "slot counts in 16 bits; two search levels of half a wavefront");
  using P = decltype(fetch(s_item[0], (int64_t)0));
  constexpr int64_t kBlock = (int64_t)kWave * U;
  for (int64_t c0 = 0; c0 < nsrc; c0 += BS) {
    int nc;
    const int64_t total = product_chunk<BS>(src, nsrc, c0, s_item, s_start, s_off, s_wave, &nc);
    // Wave w takes blocks of 64*U consecutive products; its lanes take
    // q = qb + u*64 + lane (u < U), so every load instruction is coalesced.
    for (int64_t qb = (int64_t)wave_id() * kBlock; qb < total; qb += (int64_t)NW * kBlock) {
      P p[U];
      bool ok[U];
      product_block<BS, U, Src>(s_item, s_start, s_off, nc, total, qb, fetch, p, ok);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) apply(p[u]);
    }
    block_sync();
  }
}

// A first pass over a row's products that keeps them in registers when the
// row fits one round (at most BS sources and BS*U products: one block per
// wavefront).  Then each lane's products of its wavefront's block are
// fetched with fetch_full into p[u] (ok[u] marks the valid ones), passed to
// apply1 through key(p[u]), and kept for the caller's later passes; returns
// true.  A larger row goes through for_each_product(fetch1, apply1) and
// false is returned.
template <int BS, int U, class Src, class FetchFull, class Key, class Fetch1, class Apply1, class P>
SG_DEV bool products_held(const Src& src, int64_t nsrc, typename Src::Item* s_item, int64_t* s_start, int64_t* s_off,
                          int64_t* s_wave, FetchFull& fetch_full, Key& key, Fetch1& fetch1, Apply1& apply1, P* p,
                          bool* ok) {
  constexpr int NW = BS / kWave;
  constexpr int64_t kBlock = (int64_t)kWave * U;
#pragma unroll
  for (int u = 0; u < U; ++u) ok[u] = false;
  if (nsrc <= BS) {
    int nc;
    const int64_t total = product_chunk<BS>(src, nsrc, 0, s_item, s_start, s_off, s_wave, &nc);
    if (total <= (int64_t)NW * kBlock) {
      const int64_t qb = (int64_t)wave_id() * kBlock;
      if (qb < total) {
        product_block<BS, U, Src>(s_item, s_start, s_off, nc, total, qb, fetch_full, p, ok);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (ok[u]) apply1(key(p[u]));
      }
      block_sync();
      return true;
    }
    // too many products to hold: the chunk is set up, so finish this pass
    // over it (the only chunk) here
    using P1 = decltype(fetch1(s_item[0], (int64_t)0));
    for (int64_t qb = (int64_t)wave_id() * kBlock; qb < total; qb += (int64_t)NW * kBlock) {
      P1 q[U];
      bool k[U];
      product_block<BS, U, Src>(s_item, s_start, s_off, nc, total, qb, fetch1, q, k);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k[u]) apply1(q[u]);
    }
    block_sync();
    return false;
  }
  for_each_product<BS, U>(src, nsrc, s_item, s_start, s_off, s_wave, fetch1, apply1);
  return false;
}

}  // namespace sg
