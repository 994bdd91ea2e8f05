// Semirings defined at run time (paper, Section 2.2: the user redefines the
// entry type, (+), (x) and their identities; CombBLAS and GALATIC take them
// as compile-time C++ types).
//
// A definition gives the value type and device expressions for a (+) b,
// a (x) b, the (+)-identity and the (x)-identity.  It becomes a semiring
// struct with the members the numeric kernels use -- (x) producing an
// accumulator, (+) in registers and as an atomic fold in LDS (a
// compare-and-swap loop over the value's bits), the identity that starts
// every accumulator -- and the library's own kernel templates are compiled
// for it with hipRTC: the same small-row, hash, column-slab (light and
// heavy) and whole-row tile kernels that serve the built-in semirings, for
// single products and merges.  The code object is kept per definition and
// loaded as a module on each device that uses it; the numeric launchers run
// unchanged over a kernel provider that hands out the module's functions.
#include <hip/hiprtc.h>

#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sg_handle.hpp"
#include "sg_user.hpp"

namespace sg {
namespace rtc {
extern const int kHeaderCount;
extern const char* const kHeaderNames[];
extern const char* const kHeaderTexts[];
}  // namespace rtc
}  // namespace sg

using namespace sg;

namespace {

// hipRTC has no C library headers: the two the kernel headers include are
// supplied as text (fixed-width integers come from hipRTC's own definitions).
const char* const kStdintShim =
    "#pragma once\n"
    "typedef __hip_internal::int8_t int8_t;\n"
    "typedef __hip_internal::uint8_t uint8_t;\n"
    "typedef __hip_internal::int16_t int16_t;\n"
    "typedef __hip_internal::uint16_t uint16_t;\n"
    "typedef __hip_internal::int32_t int32_t;\n"
    "typedef __hip_internal::uint32_t uint32_t;\n"
    "typedef __hip_internal::int64_t int64_t;\n"
    "typedef __hip_internal::uint64_t uint64_t;\n"
    "#define INT32_MAX 2147483647\n"
    "#define INT32_MIN (-2147483647 - 1)\n"
    "#define UINT32_MAX 4294967295u\n"
    "#define INT64_MAX 9223372036854775807ll\n"
    "#define INT64_MIN (-9223372036854775807ll - 1)\n"
    "#define UINT64_MAX 18446744073709551615ull\n";
const char* const kHipShim = "#pragma once\n";

struct VType {
  const char* name;
  int bytes;
};
const VType kTypes[] = {{"float", 4}, {"int32_t", 4}, {"uint32_t", 4}, {"double", 8}, {"int64_t", 8}, {"uint64_t", 8}};

// One kernel of a definition: its name expression and block size.
struct KName {
  std::string expr;
  int bs;
};

struct Def {
  int id = 0;
  std::string vtype;
  int vbytes = 0;
  bool idempotent = false;
  std::string key;  // the definition's text (value type, expressions, flags)
  std::vector<KName> kernels;
  std::map<std::string, std::string> lowered;
  std::vector<char> code;
  uint64_t zero_bits = 0, one_bits = 0;
  bool consts_known = false;
  struct Dev {
    hipModule_t mod = nullptr;
    std::map<std::string, KRef> fns;
  };
  std::map<int, Dev> dev;
};

std::mutex g_mu;
std::vector<std::unique_ptr<Def>> g_defs;  // id = kUserSemiringBase + index

std::string rows_product(const std::string& vt) { return "sg::OneRows<sg::SpgemmSrc<" + vt + ", true>>"; }
std::string rows_merge(const std::string& vt) { return "sg::OneRows<sg::MergeSrc<" + vt + ">>"; }

std::string n_small(const std::string& rows) { return "sg::k_num_small<sg::SrUser, " + rows + ">"; }
std::string n_hash(const std::string& rows, int lg, int bs) {
  return "sg::k_num_hash<sg::SrUser, " + rows + ", " + std::to_string(lg) + ", " + std::to_string(bs) + ">";
}
std::string n_slab(const std::string& vt, int cap, bool narrow) {
  return "sg::k_num_slab<sg::SrUser, " + vt + ", " + std::to_string(kSlabBS) + ", " + std::to_string(cap) + ", " +
         (narrow ? "true" : "false") + ">";
}
std::string n_heavy(const std::string& vt, bool narrow) {
  return "sg::k_num_slab_heavy<sg::SrUser, " + vt + ", " + std::to_string(kSlabBS) + ", " +
         (narrow ? "true" : "false") + ">";
}
std::string n_tiles(const std::string& rows, int bs) {
  return "sg::k_num_tiles<sg::SrUser, " + rows + ", " + std::to_string(bs) + ">";
}
std::string n_ranges(const std::string& rows, int lg, int bs) {
  return "sg::k_num_ranges<sg::SrUser, " + rows + ", " + std::to_string(lg) + ", " + std::to_string(bs) + ">";
}

// Host stand-in of a run-time semiring with W-sized values: the launchers
// only read the sizes of V and Acc from it (kernel arguments of V-typed
// pointers or structs have the same layout for any V of that size).
template <class W>
struct SrShape {
  using V = W;
  using Acc = W;
};

template <class W>
int item_bytes_product() {
  return (int)sizeof(typename OneRows<SpgemmSrc<W, true>>::Src::Item);
}
template <class W>
int item_bytes_merge() {
  return (int)sizeof(typename OneRows<MergeSrc<W>>::Src::Item);
}

// Every kernel the numeric launchers ask for, for single products and merges.
template <class W>
std::vector<KName> kernel_names(const std::string& vt) {
  constexpr int A = (int)sizeof(W);
  std::vector<KName> v;
  const std::string rp = rows_product(vt), rm = rows_merge(vt);
  const int ib[2] = {item_bytes_product<W>(), item_bytes_merge<W>()};
  const std::string rows[2] = {rp, rm};
  for (int m = 0; m < 2; ++m) {
    v.push_back({n_small(rows[m]), 256});
    for (int k = 0; k < kHashBins; ++k) v.push_back({n_hash(rows[m], 7 + k, hash_bs(k, A)), hash_bs(k, A)});
    v.push_back({n_tiles(rows[m], tiles_bs(A, ib[m])), tiles_bs(A, ib[m])});
    v.push_back({n_ranges(rows[m], kRangeLg, ranges_bs(A)), ranges_bs(A)});
  }
  for (bool narrow : {true, false}) {
    v.push_back({n_slab(vt, slab_cap<SrShape<W>>(), narrow), kSlabBS});
    v.push_back({n_heavy(vt, narrow), kSlabBS});
  }
  return v;
}

std::string program(const Def& d, const sg_semiring_def* def) {
  const char* word = d.vbytes == 8 ? "unsigned long long" : "unsigned int";
  std::string s;
  s += "#include \"sg_slab.hpp\"\nnamespace sg {\nstruct SrUser {\n";
  s += "  using V = " + d.vtype + ";\n  using Acc = " + d.vtype + ";\n";
  s += "  static constexpr int kId = " + std::to_string(d.id) + ";\n";
  s += "  static constexpr bool kValueMarks = false;\n";
  s += std::string("  static constexpr bool kIdempotent = ") + (d.idempotent ? "true" : "false") + ";\n";
  s += "  SG_DEV static Acc ident() { return (Acc)(" + std::string(def->zero) + "); }\n";
  s += "  SG_DEV static Acc mul(V a, V b) { return (Acc)(" + std::string(def->mul) + "); }\n";
  s += "  SG_DEV static Acc lift(V a) { return a; }\n";
  s += "  SG_DEV static Acc add(Acc a, Acc b) { return (Acc)(" + std::string(def->add) + "); }\n";
  s += "  SG_DEV static void lds_acc(Acc* p, Acc v) {\n";
  s += std::string("    using W = ") + word + ";\n";
  s += "    W* q = reinterpret_cast<W*>(p);\n";
  s += "    W old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);\n";
  s += "    while (true) {\n";
  s += "      Acc cur;\n      __builtin_memcpy(&cur, &old, sizeof(Acc));\n";
  s += "      const Acc nv = add(cur, v);\n";
  s += "      W nw;\n      __builtin_memcpy(&nw, &nv, sizeof(Acc));\n";
  s += "      if (nw == old) break;\n";
  s += "      const W seen = atomicCAS(q, old, nw);\n";
  s += "      if (seen == old) break;\n      old = seen;\n    }\n  }\n";
  s += "  SG_DEV static V out(Acc x) { return x; }\n};\n}  // namespace sg\n";
  s += "extern \"C\" __global__ void sg_user_consts(sg::SrUser::V* out) {\n";
  s += "  out[0] = sg::SrUser::ident();\n  out[1] = (sg::SrUser::V)(" + std::string(def->one) + ");\n}\n";
  return s;
}

sg_status compile(sg_handle* h, Def& d, const std::string& src) {
  std::vector<const char*> names, texts;
  for (int i = 0; i < rtc::kHeaderCount; ++i) {
    names.push_back(rtc::kHeaderNames[i]);
    texts.push_back(rtc::kHeaderTexts[i]);
  }
  names.push_back("stdint.h");
  texts.push_back(kStdintShim);
  names.push_back("hip/hip_runtime.h");
  texts.push_back(kHipShim);
  hiprtcProgram p = nullptr;
  if (hiprtcCreateProgram(&p, src.c_str(), "sg_user_semiring.hip", (int)names.size(), texts.data(), names.data()) !=
      HIPRTC_SUCCESS)
    return sg_fail(h, SG_ERR_HIP, "hiprtcCreateProgram failed");
  for (const KName& k : d.kernels) (void)hiprtcAddNameExpression(p, k.expr.c_str());
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(p, 7, opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    (void)hiprtcGetProgramLogSize(p, &n);
    std::string log(n, '\0');
    if (n) (void)hiprtcGetProgramLog(p, &log[0]);
    (void)hiprtcDestroyProgram(&p);
    if (log.size() > 4000) log.resize(4000);
    return sg_fail(h, SG_ERR_SEMIRING, "the semiring definition does not compile:\n" + log);
  }
  size_t cs = 0;
  (void)hiprtcGetCodeSize(p, &cs);
  d.code.resize(cs);
  (void)hiprtcGetCode(p, d.code.data());
  for (const KName& k : d.kernels) {
    const char* low = nullptr;
    if (hiprtcGetLoweredName(p, k.expr.c_str(), &low) != HIPRTC_SUCCESS || !low) {
      (void)hiprtcDestroyProgram(&p);
      return sg_fail(h, SG_ERR_HIP, "no compiled kernel for " + k.expr);
    }
    d.lowered[k.expr] = low;
  }
  (void)hiprtcDestroyProgram(&p);
  return SG_OK;
}

// The definition's module on h's device (loaded on first use there), and its
// identities (read once from the device).
sg_status load_on(sg_handle* h, Def& d, Def::Dev** out) {
  auto it = d.dev.find(h->device);
  if (it == d.dev.end()) {
    Def::Dev dv;
    if (hipModuleLoadData(&dv.mod, d.code.data()) != hipSuccess)
      return sg_fail(h, SG_ERR_HIP, "hipModuleLoadData failed for a run-time semiring");
    for (const KName& k : d.kernels) {
      hipFunction_t f = nullptr;
      if (hipModuleGetFunction(&f, dv.mod, d.lowered[k.expr].c_str()) != hipSuccess) {
        (void)hipModuleUnload(dv.mod);
        return sg_fail(h, SG_ERR_HIP, "hipModuleGetFunction failed for " + k.expr);
      }
      dv.fns[k.expr] = kref_module(f, k.bs);
    }
    it = d.dev.emplace(h->device, dv).first;
  }
  if (!d.consts_known) {
    hipFunction_t f = nullptr;
    void* buf = nullptr;
    if (hipModuleGetFunction(&f, it->second.mod, "sg_user_consts") != hipSuccess || hipMalloc(&buf, 16) != hipSuccess)
      return sg_fail(h, SG_ERR_HIP, "cannot evaluate the semiring's identities");
    void* args[] = {&buf};
    hipError_t e = hipModuleLaunchKernel(f, 1, 1, 1, 1, 1, 1, 0, nullptr, args, nullptr);
    uint64_t v[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(v, buf, 2 * (size_t)d.vbytes, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (e != hipSuccess) return sg_check_hip(h, e, "evaluating the semiring's identities");
    if (d.vbytes == 4) {
      uint32_t w[2];
      std::memcpy(w, v, 8);
      d.zero_bits = w[0];
      d.one_bits = w[1];
    } else {
      d.zero_bits = v[0];
      d.one_bits = v[1];
    }
    d.consts_known = true;
  }
  *out = &it->second;
  return SG_OK;
}

Def* find_def(int id) {
  const int i = id - kUserSemiringBase;
  if (i < 0 || i >= (int)g_defs.size()) return nullptr;
  return g_defs[(size_t)i].get();
}

// The module's kernels as the launchers ask for them.
template <class W>
struct KUser {
  const Def::Dev* dv;
  std::string vt;
  KRef get(const std::string& expr) const {
    auto it = dv->fns.find(expr);
    return it == dv->fns.end() ? KRef{} : it->second;
  }
  template <class Rows>
  std::string rows() const {
    if constexpr (std::is_same_v<Rows, OneRows<SpgemmSrc<W, true>>>) return rows_product(vt);
    else if constexpr (std::is_same_v<Rows, OneRows<MergeSrc<W>>>) return rows_merge(vt);
    else return std::string();
  }
  template <class Sr, class Rows>
  KRef small() const {
    return get(n_small(rows<Rows>()));
  }
  template <class Sr, class Rows, int LGS, int BS>
  KRef hash() const {
    return get(n_hash(rows<Rows>(), LGS, BS));
  }
  template <class Sr, int kCap, bool kNarrow>
  KRef slab() const {
    return get(n_slab(vt, kCap, kNarrow));
  }
  template <class Sr, bool kNarrow>
  KRef heavy() const {
    return get(n_heavy(vt, kNarrow));
  }
  template <class Sr, class Rows, int BS>
  KRef tiles() const {
    return get(n_tiles(rows<Rows>(), BS));
  }
  template <class Sr, class Rows, int LGS, int BS>
  KRef ranges() const {
    return get(n_ranges(rows<Rows>(), LGS, BS));
  }
  // (run-time semirings take the workgroup hash kernels for every hash row)
  template <class Sr, class Rows, int CAP, int BS>
  KRef merge_row() const {
    return KRef{};
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef wave_bitmap() const {
    return KRef{};
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef bitmap_row() const {
    return KRef{};
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef bitmap_dense() const {
    return KRef{};
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef ranges_bitmap() const {
    return KRef{};
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef range_runs() const {
    return KRef{};
  }
};

}  // namespace

namespace sg {

bool user_semiring(int id, int* vbytes, bool* idempotent) {
  std::lock_guard<std::mutex> lock(g_mu);
  const Def* d = find_def(id);
  if (!d) return false;
  if (vbytes) *vbytes = d->vbytes;
  if (idempotent) *idempotent = d->idempotent;
  return true;
}

sg_status user_semiring_identities(sg_handle* h, int id, uint64_t* zero_bits, uint64_t* one_bits) {
  std::lock_guard<std::mutex> lock(g_mu);
  Def* d = find_def(id);
  if (!d) return sg_fail(h, SG_ERR_SEMIRING, "unknown semiring id");
  Def::Dev* dv = nullptr;
  SG_TRY_STATUS(load_on(h, *d, &dv));
  if (zero_bits) *zero_bits = d->zero_bits;
  if (one_bits) *one_bits = d->one_bits;
  return SG_OK;
}

sg_status launch_numeric_user(sg_handle* h, const NumCtx& c, int id, hipStream_t st) {
  if (c.src.mode != kModeProduct && c.src.mode != kModeMerge)
    return sg_fail(h, SG_ERR_SEMIRING, "run-time semirings serve single products and merges, not batches");
  std::lock_guard<std::mutex> lock(g_mu);
  Def* d = find_def(id);
  if (!d) return sg_fail(h, SG_ERR_SEMIRING, "unknown semiring id");
  Def::Dev* dv = nullptr;
  SG_TRY_STATUS(load_on(h, *d, &dv));
  if (d->vbytes == 4) launch_numeric<SrShape<uint32_t>, SrShape<uint32_t>>(c, st, KUser<uint32_t>{dv, d->vtype});
  else launch_numeric<SrShape<uint64_t>, SrShape<uint64_t>>(c, st, KUser<uint64_t>{dv, d->vtype});
  return SG_OK;
}

}  // namespace sg

extern "C" {

sg_status sg_semiring_define(sg_handle* h, const sg_semiring_def* def, sg_semiring* out) {
  if (!h || !out) return SG_ERR_INVALID;
  if (!def || !def->value_type || !def->add || !def->mul || !def->zero || !def->one)
    return sg_fail(h, SG_ERR_INVALID, "a semiring definition needs a value type, (+), (x), zero and one");
  if (def->flags & ~(uint32_t)SG_SR_IDEMPOTENT) return sg_fail(h, SG_ERR_INVALID, "unknown semiring flag");
  const VType* vt = nullptr;
  for (const VType& t : kTypes)
    if (std::strcmp(def->value_type, t.name) == 0) vt = &t;
  if (!vt)
    return sg_fail(h, SG_ERR_INVALID,
                   "value_type must be float, double, int32_t, uint32_t, int64_t or uint64_t");
  if (hipSetDevice(h->device) != hipSuccess) return sg_fail(h, SG_ERR_HIP, "hipSetDevice failed");
  const std::string key = std::string(def->value_type) + '\x1f' + def->add + '\x1f' + def->mul + '\x1f' + def->zero +
                          '\x1f' + def->one + '\x1f' + std::to_string(def->flags);
  std::lock_guard<std::mutex> lock(g_mu);
  Def* d = nullptr;
  for (auto& p : g_defs)
    if (p->key == key) d = p.get();
  if (!d) {
    if (kUserSemiringBase + (int)g_defs.size() > INT32_MAX - 1) return sg_fail(h, SG_ERR_INVALID, "too many semirings");
    auto nd = std::make_unique<Def>();
    nd->id = kUserSemiringBase + (int)g_defs.size();
    nd->vtype = vt->name;
    nd->vbytes = vt->bytes;
    nd->idempotent = (def->flags & SG_SR_IDEMPOTENT) != 0;
    nd->key = key;
    nd->kernels = vt->bytes == 4 ? kernel_names<uint32_t>(vt->name) : kernel_names<uint64_t>(vt->name);
    SG_TRY_STATUS(compile(h, *nd, program(*nd, def)));
    g_defs.push_back(std::move(nd));
    d = g_defs.back().get();
  }
  Def::Dev* dv = nullptr;
  SG_TRY_STATUS(load_on(h, *d, &dv));
  out->id = d->id;
  out->value_bytes = d->vbytes;
  out->acc_flags = SG_ACC_DEFAULT;
  out->comp_min_terms = 64;
  out->comp_min_products = 0;
  return SG_OK;
}

}  // extern "C"
