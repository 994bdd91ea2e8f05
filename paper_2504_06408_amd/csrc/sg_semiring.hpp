// Device-side semirings (paper, Section 2.2): value type V, the accumulator
// type Acc kept in LDS, the identity of (+) used to initialise accumulator
// slots, (x) producing an Acc, (+) on Acc both atomically in LDS and in
// registers, and the final conversion back to V.  kIdempotent: x (+) x = x,
// so folding a product twice equals folding it once.
//
// Slots start at the (+)-identity, so "0 (+) first product" stands in for
// "first product initialises the slot"; the two agree exactly except for the
// sign of a float zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_device.hpp"

namespace sg {

// (+, x) over int64 with wrap-around modulo 2^64.
struct SrI64 {
  using V = int64_t;
  using Acc = unsigned long long;
  static constexpr int kId = 1;
  static constexpr bool kValueMarks = false;
  static constexpr bool kIdempotent = false;
  SG_DEV static Acc ident() { return 0ull; }
  SG_DEV static Acc mul(V a, V b) { return (Acc)a * (Acc)b; }
  SG_DEV static Acc lift(V a) { return (Acc)a; }
  SG_DEV static Acc add(Acc x, Acc y) { return x + y; }
  SG_DEV static void lds_acc(Acc* p, Acc v) { atomicAdd(p, v); }
  SG_DEV static V out(Acc x) { return (V)x; }
};

// (+, x) over binary32, plain accumulation.
struct SrF32 {
  using V = float;
  using Acc = float;
  static constexpr int kId = 2;
  static constexpr bool kValueMarks = false;
  static constexpr bool kIdempotent = false;
  SG_DEV static Acc ident() { return 0.0f; }
  SG_DEV static Acc mul(V a, V b) { return a * b; }
  SG_DEV static Acc lift(V a) { return a; }
  SG_DEV static Acc add(Acc x, Acc y) { return x + y; }
  SG_DEV static void lds_acc(Acc* p, Acc v) { atomicAdd(p, v); }
  SG_DEV static V out(Acc x) { return x; }
};

// (+, x) over binary32 with compensated accumulation: each slot holds a
// float pair (hi, lo).  A product enters as (p, e) with p = fl(a*b) and e its
// exact rounding error (one FMA, the "TwoProduct" of Ogita, Rump and Oishi,
// SIAM J. Sci. Comput. 2005); adding it to a slot takes Knuth's TwoSum of hi
// and p and folds both error terms into lo.  The result is hi + lo rounded
// once.  The pair is updated with a 64-bit compare-and-swap in LDS.
struct SrF32Comp {
  using V = float;
  using Acc = unsigned long long;  // low word: hi, high word: lo
  static constexpr int kId = 2;
  static constexpr bool kValueMarks = false;
  static constexpr bool kIdempotent = false;
  SG_DEV static Acc pack(float hi, float lo) {
    return (Acc)__float_as_uint(hi) | ((Acc)__float_as_uint(lo) << 32);
  }
  SG_DEV static float hi_of(Acc x) { return __uint_as_float((uint32_t)x); }
  SG_DEV static float lo_of(Acc x) { return __uint_as_float((uint32_t)(x >> 32)); }
  SG_DEV static void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
  }
  SG_DEV static Acc ident() { return 0ull; }
  SG_DEV static Acc mul(V a, V b) {
    const float p = a * b;
    const float e = __builtin_fmaf(a, b, -p);
    return pack(p, e);
  }
  SG_DEV static Acc lift(V a) { return pack(a, 0.0f); }
  SG_DEV static Acc add(Acc x, Acc y) {
    float s, e;
    two_sum(hi_of(x), hi_of(y), s, e);
    return pack(s, lo_of(x) + (lo_of(y) + e));
  }
  SG_DEV static void lds_acc(Acc* p, Acc v) {
    Acc old = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (true) {
      const Acc nv = add(old, v);
      const Acc seen = atomicCAS(p, old, nv);
      if (seen == old) break;
      old = seen;
    }
  }
  SG_DEV static V out(Acc x) { return hi_of(x) + lo_of(x); }
};

// (+, x) over binary64.
struct SrF64 {
  using V = double;
  using Acc = double;
  static constexpr int kId = 3;
  static constexpr bool kValueMarks = false;
  static constexpr bool kIdempotent = false;
  SG_DEV static Acc ident() { return 0.0; }
  SG_DEV static Acc mul(V a, V b) { return a * b; }
  SG_DEV static Acc lift(V a) { return a; }
  SG_DEV static Acc add(Acc x, Acc y) { return x + y; }
  SG_DEV static void lds_acc(Acc* p, Acc v) { atomicAdd(p, v); }
  SG_DEV static V out(Acc x) { return x; }
};

// (or, and) over uint8 truth values.  An LDS slot only ever goes 0 -> 1, so a
// plain byte store of 1 is a race-free "atomic or".
struct SrBool {
  using V = uint8_t;
  using Acc = uint8_t;
  static constexpr int kId = 4;
  static constexpr bool kValueMarks = false;
  static constexpr bool kIdempotent = true;
  SG_DEV static Acc ident() { return 0; }
  SG_DEV static Acc mul(V a, V b) { return (a != 0 && b != 0) ? 1 : 0; }
  SG_DEV static Acc lift(V a) { return a != 0 ? 1 : 0; }
  SG_DEV static Acc add(Acc x, Acc y) { return (x | y) ? 1 : 0; }
  SG_DEV static void lds_acc(Acc* p, Acc v) {
    if (v) __hip_atomic_store(p, (Acc)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  SG_DEV static V out(Acc x) { return x; }
};

// (min, +) over binary32.  Accumulators hold an order-preserving unsigned
// image of the float (negative values bit-inverted, non-negative ones with
// the sign bit set), so the minimum is a single integer atomic min.  The
// identity 0xFFFFFFFF lies above the image of +inf.  No product maps to the
// identity, so a slot that still holds it was never reached (kValueMarks):
// dense accumulators need no separate occupancy bitmap.
struct SrMinPlus {
  using V = float;
  using Acc = uint32_t;
  static constexpr int kId = 5;
  static constexpr bool kValueMarks = true;
  static constexpr bool kIdempotent = true;
  SG_DEV static uint32_t key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  }
  SG_DEV static float unkey(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
  }
  SG_DEV static Acc ident() { return 0xFFFFFFFFu; }
  SG_DEV static Acc mul(V a, V b) { return key(a + b); }
  SG_DEV static Acc lift(V a) { return key(a); }
  SG_DEV static Acc add(Acc x, Acc y) { return x < y ? x : y; }
  SG_DEV static void lds_acc(Acc* p, Acc v) { atomicMin(p, v); }
  SG_DEV static V out(Acc x) { return unkey(x); }
};

}  // namespace sg
