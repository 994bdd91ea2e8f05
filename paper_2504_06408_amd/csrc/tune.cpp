// Autotuner and tuning tables.
//
// Two thresholds decide which accumulator a row or tile gets:
//   hash_max_products  rows with more products leave the LDS-hash path for the
//                      column-tiled dense path (bitmap symbolic, task numeric);
//   dense_tile_min     a dense row's tile with at least this many entries gets
//                      a dense LDS accumulator (no sort); sparser tiles are
//                      grouped into hash range tasks (radix sort).
// sg_tune times the whole two-pass product for each pair of candidates with
// HIP events (best of two timed runs after a warm-up) and keeps the fastest.
// A table is a small JSON object:
//   {"hash_max_products": N, "dense_tile_min": M, "semiring": id,
//    "timings_ms": {"N/M": ms, ...}}
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
  long long t = 0;
  if (find_int(s, "dense_tile_min", &t)) {
    if (t < 1 || t > sg::kRangeCap) return sg_fail(h, SG_ERR_INVALID, "tuning table has a bad dense_tile_min");
    h->tile_min = (int32_t)t;
  }
  h->cache_valid = false;
  return SG_OK;
}

sg_status sg_tune(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, const char* out_json) {
  if (!h || !sr || !A || !B || !out_json) return SG_ERR_INVALID;
  const int64_t keep_hm = h->hash_max;
  const int32_t keep_tm = h->tile_min;
  const int keep_force = h->force;
  h->force = sg::kForceAuto;
  static const int64_t cand_hm[] = {256, 1024, 4096};
  static const int32_t cand_tm[] = {512, 1024, 2048};
  std::vector<double> ms;
  int64_t best_hm = keep_hm;
  int32_t best_tm = keep_tm;
  double best_ms = 1e300;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SG_ERR_HIP;
  int64_t* rowptr = nullptr;
  void* buf = nullptr;
  size_t buf_cap = 0;
  sg_status st = SG_OK;
  if (hipMalloc(&rowptr, sizeof(int64_t) * (size_t)(A->nrows + 1)) != hipSuccess) st = SG_ERR_NOMEM;
  for (int64_t hm : cand_hm) {
    for (int32_t tm : cand_tm) {
      if (st != SG_OK) break;
      h->hash_max = hm;
      h->tile_min = tm;
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
        if (rep > 0 && t < t_best) t_best = t;  // the first run warms up
      }
      ms.push_back(t_best);
      if (t_best < best_ms) {
        best_ms = t_best;
        best_hm = hm;
        best_tm = tm;
      }
    }
  }
  if (rowptr) (void)hipFree(rowptr);
  if (buf) (void)hipFree(buf);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->force = keep_force;
  h->cache_valid = false;
  if (st != SG_OK) {
    h->hash_max = keep_hm;
    h->tile_min = keep_tm;
    return st;
  }
  h->hash_max = best_hm;
  h->tile_min = best_tm;
  FILE* f = std::fopen(out_json, "w");
  if (!f) return sg_fail(h, SG_ERR_INVALID, std::string("cannot write ") + out_json);
  std::fprintf(f, "{\n  \"hash_max_products\": %lld,\n  \"dense_tile_min\": %d,\n  \"semiring\": %d,\n  \"timings_ms\": {",
               (long long)best_hm, (int)best_tm, sr->id);
  size_t k = 0;
  for (int64_t hm : cand_hm)
    for (int32_t tm : cand_tm) {
      std::fprintf(f, "%s\"%lld/%d\": %.4f", k ? ", " : "", (long long)hm, (int)tm, ms[k]);
      ++k;
    }
  std::fprintf(f, "}\n}\n");
  std::fclose(f);
  return SG_OK;
}

}  // extern "C"
