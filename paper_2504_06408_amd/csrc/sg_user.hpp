// Semirings defined at run time (user_sr.cpp): lookup and numeric launch.
#pragma once

#include "sg_handle.hpp"

#define SG_TRY_STATUS(expr)         \
  do {                              \
    const sg_status _s = (expr);    \
    if (_s != SG_OK) return _s;     \
  } while (0)

namespace sg {

// Ids of run-time semirings start here (the built-in ones are 1..5).
constexpr int kUserSemiringBase = 64;

// Whether id names a defined run-time semiring; its value width and whether
// its (+) is idempotent.
bool user_semiring(int id, int* vbytes, bool* idempotent);
// The value bits of its (+)- and (x)-identities (loads its module on h's
// device if needed).
sg_status user_semiring_identities(sg_handle* h, int id, uint64_t* zero_bits, uint64_t* one_bits);
// The numeric pass of c (a single product or merge) with its kernels.
sg_status launch_numeric_user(sg_handle* h, const NumCtx& c, int id, hipStream_t st);

}  // namespace sg
