// Autotuner and tuning tables (paper, Section 4.3: the local multiply's
// library exposes tunable parameters; Section 5.1 reports that tuning them
// changed little on the paper's inputs -- here the choice is measured on the
// caller's own product).
//
// The knobs are the ones the default path reads:
//   hash_max_products  rows with more products leave the LDS-hash path for the
//                      column-slab dense path;
//   slab_log           the dense path's slab width 2^slab_log columns (14..17;
//                      wider slabs mean fewer, larger tasks per dense row);
//   light_cap          a dense row's slab with at most this many output
//                      entries is one light task (bitmap and ranks in LDS),
//                      a fuller slab a heavy one (a dense LDS accumulator per
//                      column tile); the largest useful value is the light
//                      kernel's LDS capacity for the semiring's accumulator.
// sg_tune times the whole two-pass product (symbolic with its read-back, then
// numeric) with HIP events, best of two timed runs after a warm-up, and walks
// the knobs one at a time (coordinate descent from the defaults, repeated
// while a sweep still improves, at most three sweeps).
//
// A table is a JSON object for one semiring and value width:
//   {"semiring": id, "value_bytes": b, "acc_flags": f, "hash_max_products": N,
//    "slab_log": L, "light_cap": C, "default_ms": t0, "tuned_ms": t1,
//    "timings_ms": {"N/L/C": ms, ...}}
// hash_max_products and slab_log shape the structure (the symbolic pass,
// which knows no semiring) and apply to every product of the handle;
// light_cap is kept for the table's semiring only.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "sg_handle.hpp"

namespace {

bool find_int(const std::string& s, const char* key, long long* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) return false;
  p = s.find(':', p + k.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < s.size() && (s[p] == ' ' || s[p] == '\t' || s[p] == '\n' || s[p] == '\r')) ++p;
  char* end = nullptr;
  const long long v = std::strtoll(s.c_str() + p, &end, 10);
  if (end == s.c_str() + p) return false;
  *out = v;
  return true;
}

// LDS capacity of a light task for the accumulator the semiring's dense rows
// use (accumulators and 16-bit columns in 42 KB; compensated fp32 sums keep a
// float pair).
int32_t full_light_cap(const sg_semiring* sr) {
  int acc = sr->value_bytes;
  if (sr->id == SG_PLUS_TIMES_F32 && sr->acc_flags != SG_ACC_PLAIN) acc = 8;
  return sg::light_cap_of(acc);
}

struct Knobs {
  int64_t hm;
  int32_t ls, cap;
  bool operator<(const Knobs& o) const { return std::tie(hm, ls, cap) < std::tie(o.hm, o.ls, o.cap); }
};

}  // namespace

extern "C" {

sg_status sg_tune_load(sg_handle* h, const sg_semiring* sr, const char* path) {
  if (!h || !path) return SG_ERR_INVALID;
  std::ifstream f(path);
  if (!f) return sg_fail(h, SG_ERR_INVALID, std::string("cannot read tuning table ") + path);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  long long sid = 0, vb = 0, hm = 0, ls = 0, cap = 0;
  if (!find_int(s, "semiring", &sid) || sid < 1 || sid > 5 || !find_int(s, "value_bytes", &vb))
    return sg_fail(h, SG_ERR_INVALID, "tuning table lacks its semiring id and value width");
  if (sr && (sr->id != sid || sr->value_bytes != vb))
    return sg_fail(h, SG_ERR_SEMIRING, "the tuning table was made for semiring " + std::to_string(sid) + " (" +
                                           std::to_string(vb) + "-byte values), not for semiring " +
                                           std::to_string(sr->id));
  if (!find_int(s, "hash_max_products", &hm) || hm < 0 || hm > sg::kHashCap)
    return sg_fail(h, SG_ERR_INVALID, "tuning table lacks a valid hash_max_products");
  if (find_int(s, "slab_log", &ls) && ls != 0 && (ls < sg::kSlabLogMin || ls > sg::kSlabLogMax))
    return sg_fail(h, SG_ERR_INVALID, "tuning table has a bad slab_log");
  if (find_int(s, "light_cap", &cap) && (cap < 0 || cap > 32768))
    return sg_fail(h, SG_ERR_INVALID, "tuning table has a bad light_cap");
  long long t = 0;
  if (find_int(s, "dense_tile_min", &t)) {
    if (t < 1 || t > sg::kRangeCap) return sg_fail(h, SG_ERR_INVALID, "tuning table has a bad dense_tile_min");
    h->tile_min = (int32_t)t;
  }
  h->hash_max = hm;
  h->slab_ls = (int32_t)ls;
  h->light_cap = (int32_t)cap;
  h->tuned_sr = (int32_t)sid;
  h->tuned_vb = (int32_t)vb;
  h->cache_valid = false;
  return SG_OK;
}

sg_status sg_tune(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, const char* out_json) {
  if (!h || !sr || !A || !B || !out_json) return SG_ERR_INVALID;
  if (sr->id < 1 || sr->id > 5) return sg_fail(h, SG_ERR_SEMIRING, "unknown semiring id");
  const int64_t keep_hm = h->hash_max;
  const int32_t keep_ls = h->slab_ls, keep_cap = h->light_cap, keep_tsr = h->tuned_sr, keep_tvb = h->tuned_vb;
  const int keep_force = h->force;
  h->force = sg::kForceAuto;
  // the candidates of each knob (the defaults first)
  const int32_t ls0 = sg::slab_log(B->ncols);
  std::vector<int64_t> c_hm = {sg::kHashCap, 2048, 1024};
  std::vector<int32_t> c_ls = {ls0};
  if (ls0 - 1 >= sg::kSlabLogMin) c_ls.push_back(ls0 - 1);
  if (ls0 + 1 <= sg::kSlabLogMax) c_ls.push_back(ls0 + 1);
  const int32_t full = full_light_cap(sr);
  std::vector<int32_t> c_cap = {full, full / 2, full / 4};
  std::map<Knobs, double> ms;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int64_t* rowptr = nullptr;
  void* buf = nullptr;
  size_t buf_cap = 0;
  sg_status st = SG_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = SG_ERR_HIP;
  if (st == SG_OK && hipMalloc(&rowptr, sizeof(int64_t) * (size_t)(A->nrows + 1)) != hipSuccess) st = SG_ERR_NOMEM;
  // whole two-pass product time of one setting (cached)
  auto time_of = [&](const Knobs& k) -> double {
    auto it = ms.find(k);
    if (it != ms.end()) return it->second;
    h->hash_max = k.hm;
    h->slab_ls = k.ls;
    h->light_cap = k.cap;
    h->tuned_sr = 0;
    h->cache_valid = false;
    double t_best = 1e300;
    for (int rep = 0; rep < 3 && st == SG_OK; ++rep) {
      (void)hipEventRecord(e0, nullptr);
      int64_t nnz = 0;
      st = sg_spgemm_symbolic(h, A, B, rowptr, &nnz, nullptr);
      if (st != SG_OK) break;
      const size_t need = (size_t)nnz * (4 + (size_t)sr->value_bytes) + 512;
      if (need > buf_cap) {
        if (buf) (void)hipFree(buf);
        buf = nullptr;
        buf_cap = 0;
        if (hipMalloc(&buf, need) != hipSuccess) {
          st = sg_fail(h, SG_ERR_NOMEM, "sg_tune: no device memory for the product");
          break;
        }
        buf_cap = need;
      }
      sg_csr C{A->nrows, B->ncols, nnz, rowptr, (int32_t*)buf, (char*)buf + (((size_t)nnz * 4 + 255) & ~(size_t)255)};
      st = sg_spgemm_numeric(h, sr, A, B, &C, nullptr);
      (void)hipEventRecord(e1, nullptr);
      (void)hipEventSynchronize(e1);
      float t = 0;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (rep > 0 && t < t_best) t_best = t;  // the first run warms up
    }
    ms[k] = t_best;
    return t_best;
  };
  Knobs best{c_hm[0], c_ls[0], c_cap[0]};
  const double t_default = st == SG_OK ? time_of(best) : 1e300;
  double t_best = t_default;
  for (int sweep = 0; sweep < 3 && st == SG_OK; ++sweep) {
    const Knobs before = best;
    for (int64_t v : c_hm) {
      const Knobs k{v, best.ls, best.cap};
      const double t = time_of(k);
      if (st == SG_OK && t < t_best) {
        t_best = t;
        best = k;
      }
    }
    for (int32_t v : c_ls) {
      const Knobs k{best.hm, v, best.cap};
      const double t = time_of(k);
      if (st == SG_OK && t < t_best) {
        t_best = t;
        best = k;
      }
    }
    for (int32_t v : c_cap) {
      const Knobs k{best.hm, best.ls, v};
      const double t = time_of(k);
      if (st == SG_OK && t < t_best) {
        t_best = t;
        best = k;
      }
    }
    if (!(before < best) && !(best < before)) break;
  }
  if (rowptr) (void)hipFree(rowptr);
  if (buf) (void)hipFree(buf);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->force = keep_force;
  h->cache_valid = false;
  if (st != SG_OK) {
    h->hash_max = keep_hm;
    h->slab_ls = keep_ls;
    h->light_cap = keep_cap;
    h->tuned_sr = keep_tsr;
    h->tuned_vb = keep_tvb;
    return st;
  }
  h->hash_max = best.hm;
  h->slab_ls = best.ls;
  h->light_cap = best.cap;
  h->tuned_sr = sr->id;
  h->tuned_vb = sr->value_bytes;
  FILE* f = std::fopen(out_json, "w");
  if (!f) return sg_fail(h, SG_ERR_INVALID, std::string("cannot write ") + out_json);
  std::fprintf(f,
               "{\n  \"semiring\": %d,\n  \"value_bytes\": %d,\n  \"acc_flags\": %u,\n  \"hash_max_products\": %lld,\n"
               "  \"slab_log\": %d,\n  \"light_cap\": %d,\n  \"default_ms\": %.4f,\n  \"tuned_ms\": %.4f,\n"
               "  \"timings_ms\": {",
               sr->id, sr->value_bytes, sr->acc_flags, (long long)best.hm, best.ls, best.cap, t_default, t_best);
  size_t k = 0;
  for (const auto& kv : ms) {
    std::fprintf(f, "%s\"%lld/%d/%d\": %.4f", k ? ", " : "", (long long)kv.first.hm, kv.first.ls, kv.first.cap,
                 kv.second);
    ++k;
  }
  std::fprintf(f, "}\n}\n");
  std::fclose(f);
  return SG_OK;
}

}  // extern "C"
