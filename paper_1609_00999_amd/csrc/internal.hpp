// internal.hpp -- host-side helpers shared by the libmont translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mont.h"

namespace mont {

// Validate a parameter block handed in by a caller: it must be what
// mont_setup produces for its modulus (odd 3 <= P < 2^31, P*P' = -1 mod 2^32).
inline bool params_ok(const mont_params* prm) {
  if (!prm) return false;
  uint32_t P = prm->P;
  if (P < 3 || (P & 1u) == 0 || P >= 0x80000000u) return false;
  if ((uint32_t)(P * prm->Pprime) != 0xFFFFFFFFu) return false;
  if (prm->R1 >= P || prm->R2 >= P) return false;
  return true;
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Map the last launch error to a status.
inline mont_status last_launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MONT_OK : MONT_EHIP;
}

// Launch shape of the streaming elementwise kernels.
struct ElemTune {
  int block;  // threads per workgroup: 256 or 512
  int vpt;    // 128-bit vectors per thread per pass: 1, 2 or 4
  int nt;     // 1 = non-temporal loads and stores
};

enum ElemOp { OP_TO = 0, OP_FROM = 1, OP_MUL = 2, OP_MULADD = 3, OP_POW = 4, OP_MODMUL = 5, OP_COUNT = 6 };

ElemTune& elem_tune(int op);

}  // namespace mont
