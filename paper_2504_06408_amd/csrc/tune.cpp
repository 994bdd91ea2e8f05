// Autotuner and tuning tables.
//
// The tunable is the product count above which a row leaves the LDS hash
// path for the column-tiled dense path (the hash path needs a sort, the dense
// path pays per-tile fixed costs).  sg_tune times the whole two-pass product
// for each candidate with HIP events and keeps the fastest.  A table is a
// small JSON object: {"hash_max_products": N, "semiring": id, "timings_ms": {...}}.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
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

}  // namespace

extern "C" {

sg_status sg_tune_load(sg_handle* h, const char* path) {
  std::ifstream f(path);
  if (!f) return sg_fail(h, SG_ERR_INVALID, std::string("cannot read tuning table ") + path);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  long long v = 0;
  if (!find_int(s, "hash_max_products", &v) || v < 0 || v > sg::kHashCap)
    return sg_fail(h, SG_ERR_INVALID, "tuning table lacks a valid hash_max_products");
  h->hash_max = v;
  h->cache_valid = false;
  return SG_OK;
}

sg_status sg_tune(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, const char* out_json) {
  if (!h || !sr || !A || !B || !out_json) return SG_ERR_INVALID;
  const int64_t keep = h->hash_max;
  const int keep_force = h->force;
  h->force = sg::kForceAuto;
  static const int64_t cand[] = {64, 256, 512, 1024, 2048, 4096};
  std::vector<double> ms;
  int64_t best = keep;
  double best_ms = 1e300;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SG_ERR_HIP;
  int64_t* rowptr = nullptr;
  void* buf = nullptr;
  size_t buf_cap = 0;
  sg_status st = SG_OK;
  if (hipMalloc(&rowptr, sizeof(int64_t) * (size_t)(A->nrows + 1)) != hipSuccess) st = SG_ERR_NOMEM;
  for (int64_t hm : cand) {
    if (st != SG_OK) break;
    h->hash_max = hm;
    h->cache_valid = false;
    double t_best = 1e300;
    for (int rep = 0; rep < 3 && st == SG_OK; ++rep) {
      (void)hipEventRecord(e0, nullptr);
      int64_t nnz = 0;
      st = sg_spgemm_symbolic(h, A, B, rowptr, &nnz, nullptr);
      if (st != SG_OK) break;
      const size_t need = (size_t)nnz * (4 + (size_t)sr->value_bytes) + 256;
      if (need > buf_cap) {
        if (buf) (void)hipFree(buf);
        buf = nullptr;
        if (hipMalloc(&buf, need) != hipSuccess) {
          st = SG_ERR_NOMEM;
          break;
        }
        buf_cap = need;
      }
      sg_csr C{A->nrows, B->ncols, nnz, rowptr, (int32_t*)buf,
               (char*)buf + (((size_t)nnz * 4 + 255) & ~(size_t)255)};
      st = sg_spgemm_numeric(h, sr, A, B, &C, nullptr);
      (void)hipEventRecord(e1, nullptr);
      (void)hipEventSynchronize(e1);
      float t = 0;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (rep > 0 && t < t_best) t_best = t;  // first repetition warms up
    }
    ms.push_back(t_best);
    if (t_best < best_ms) {
      best_ms = t_best;
      best = hm;
    }
  }
  if (rowptr) (void)hipFree(rowptr);
  if (buf) (void)hipFree(buf);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->force = keep_force;
  h->cache_valid = false;
  if (st != SG_OK) {
    h->hash_max = keep;
    return st;
  }
  h->hash_max = best;
  FILE* f = std::fopen(out_json, "w");
  if (!f) return sg_fail(h, SG_ERR_INVALID, std::string("cannot write ") + out_json);
  std::fprintf(f, "{\n  \"hash_max_products\": %lld,\n  \"semiring\": %d,\n  \"timings_ms\": {", (long long)best,
               sr->id);
  for (size_t i = 0; i < ms.size(); ++i)
    std::fprintf(f, "%s\"%lld\": %.4f", i ? ", " : "", (long long)cand[i], ms[i]);
  std::fprintf(f, "}\n}\n");
  std::fclose(f);
  return SG_OK;
}

}  // extern "C"
