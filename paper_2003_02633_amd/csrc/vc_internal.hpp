// vc_internal.hpp -- host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vc.h"
#include "../../include/vc_device.hpp"
#include "vc_params.hpp"

namespace vc {

// launch configuration of the streaming axpy (chosen by the autotuner, paper_2003_02633_amd/tune.py)
struct StreamCfg {
  int block;       // threads per block
  int vpt;         // pairs of codes per lane and grid step (1, 2, or 4 with 256 or 512 threads)
  int nt;          // non-temporal loads/stores
};
StreamCfg stream_cfg(int prec);                                   // prec: PREC_F32 / PREC_F64
vc_status set_axpy_cfg(int prec, int block, int vpt, int nt);     // prec -1: both

vc_status launch_encode(const Resolved& R, const float* xyz, uint64_t* codes, size_t n, hipStream_t s);
vc_status launch_decode(const Resolved& R, const uint64_t* codes, float* xyz, size_t n, hipStream_t s);
vc_status launch_axpy(const Resolved& R, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* c,
                      size_t n, float* c32_dump, hipStream_t s);
vc_status launch_dot(const Resolved& R, const uint64_t* a, const uint64_t* b, size_t n, float* partials,
                     int nparts, float* d_out, hipStream_t s);
vc_status launch_norm2(const Resolved& R, const uint64_t* a, size_t n, float* partials, int nparts,
                       float* d_out, hipStream_t s);
int reduce_parts(size_t n);
vc_status launch_apply(const Resolved& R, const float* M, int rows, int cols, const uint64_t* U, float* out,
                       size_t n_elem, hipStream_t s);

inline vc_status launch_status()
{
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? VC_SUCCESS : VC_ERROR_LAUNCH;
}

// layout x mode x precision dispatch (decode-only paths ignore the precision and the
// magnitude rounding); the truncating magnitude of the 22-bit mantissa is keys 16-19
#define VC_CASES(FN, PR, ...)                                                             \
  case 0: return FN<L0722, PLAIN, PR>(__VA_ARGS__);                                       \
  case 1: return FN<L0722, TANH, PR>(__VA_ARGS__);                                        \
  case 2: return FN<L0722, COS, PR>(__VA_ARGS__);                                         \
  case 3: return FN<L0722, FRAC, PR>(__VA_ARGS__);                                        \
  case 4: return FN<L0723, PLAIN, PR>(__VA_ARGS__);                                       \
  case 8: return FN<L0823, PLAIN, PR>(__VA_ARGS__);                                       \
  case 12: return FN<L1823, PLAIN, PR>(__VA_ARGS__);
#define VC_CASES_TRUNC(FN, PR, ...)                                                       \
  case 16: return FN<L0722T, PLAIN, PR>(__VA_ARGS__);                                     \
  case 17: return FN<L0722T, TANH, PR>(__VA_ARGS__);                                      \
  case 18: return FN<L0722T, COS, PR>(__VA_ARGS__);                                       \
  case 19: return FN<L0722T, FRAC, PR>(__VA_ARGS__);
#define VC_ENC_KEY(R) ((R).layout * 4 + (R).mode + ((R).mag_round == VC_MAG_TRUNC ? 16 : 0))
#define VC_DISPATCH(R, FN, ...)                                                           \
  do {                                                                                    \
    if ((R).prec == PREC_F64) {                                                           \
      switch (VC_ENC_KEY(R)) {                                                            \
        VC_CASES(FN, PREC_F64, __VA_ARGS__)                                               \
        VC_CASES_TRUNC(FN, PREC_F64, __VA_ARGS__)                                         \
        default: return VC_ERROR_UNSUPPORTED_CODEC;                                       \
      }                                                                                   \
    } else {                                                                              \
      switch (VC_ENC_KEY(R)) {                                                            \
        VC_CASES(FN, PREC_F32, __VA_ARGS__)                                               \
        VC_CASES_TRUNC(FN, PREC_F32, __VA_ARGS__)                                         \
        default: return VC_ERROR_UNSUPPORTED_CODEC;                                       \
      }                                                                                   \
    }                                                                                     \
  } while (0)
#define VC_DISPATCH_NOPREC(R, FN, ...)                                                    \
  do {                                                                                    \
    switch ((R).layout * 4 + (R).mode) {                                                  \
      VC_CASES(FN, PREC_F32, __VA_ARGS__)                                                 \
      default: return VC_ERROR_UNSUPPORTED_CODEC;                                         \
    }                                                                                     \
  } while (0)

}  // namespace vc
