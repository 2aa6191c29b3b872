/*
 * vc_inline.hpp -- the codec as device functions, for encoding and decoding 3-vectors inside the
 * caller's own HIP kernels (gfx950).  This is the inline use the method is designed for (§1):
 * a kernel keeps its vectors compressed in HBM and converts them in registers where it reads or
 * writes them, as the flux-divergence kernel of Alg. (fr_fdiv_comp) does with its flux rows.
 *
 * Host side (libvc, vc_ext.h):
 *     vc_codec c;  vc_codec_init(&c, "0,7,22-17-18");        // or any codec the library accepts
 *     vc_inline::Params p;
 *     vcx_inline_params(&c, &p, sizeof p);                   // resolved constants, host memory
 *     my_kernel<<<grid, block>>>(..., p);                     // passed by value
 * Device side:
 *     uint64_t w = vc_inline::encode(p, x, y, z);            // Eq. (a_disc), §2.3 magnitude
 *     vc_inline::decode(p, w, x, y, z);                      // Eq. (a_inv), Eq. (cart2sphere)
 *     float d = vc_inline::dot(p, wa, wb);                   // decode(wa) . decode(wb)
 * The template arguments select the layout (vc_inline::L0722, L0723, L0823, L1823; L0722T for
 * the <0,7,22> layout with VC_MAG_TRUNC, where the other layouts' truncation equals nearest-even),
 * the mode (PLAIN, TANH, COS, FRAC) and the encoder precision (PREC_F64, PREC_F32); they must
 * match the codec given to vcx_inline_params (the defaults match vc_codec_init's defaults).  The results
 * are those of the library's own kernels, bit for bit: both compile the same functions.
 *
 * Build user kernels with hipcc --offload-arch=gfx950 -Xclang -target-feature -Xclang
 * -packed-fp32-ops (the flags the library is built with) and this directory on the include path.
 */
#pragma once

#include <stdint.h>

#include "vc_device.hpp"

namespace vc_inline {

using Params = vc::Params;
using L0722 = vc::L0722;
using L0723 = vc::L0723;
using L0823 = vc::L0823;
using L1823 = vc::L1823;
using L0722T = vc::L0722T;   // <0,7,22>-17-18 with the truncating magnitude (VC_MAG_TRUNC)
constexpr int PLAIN = vc::PLAIN, TANH = vc::TANH, COS = vc::COS, FRAC = vc::FRAC;
constexpr int PREC_F32 = vc::PREC_F32, PREC_F64 = vc::PREC_F64;

/* The 64-bit code of (x, y, z); non-finite input gives the reserved code, the zero vector 0. */
template <class L = L0722, int MODE = PLAIN, int PREC = PREC_F64>
__device__ __forceinline__ uint64_t encode(const Params& P, float x, float y, float z)
{
  return vc::encode_vec<L, MODE, PREC>(x, y, z, P);
}

/* The float32 vector of a code (NaN components for the reserved code). */
template <class L = L0722, int MODE = PLAIN>
__device__ __forceinline__ void decode(const Params& P, uint64_t w, float& x, float& y, float& z)
{
  vc::decode_vec<L, MODE>(w, P, x, y, z);
}

/* |decode(w)|, from the exponent and mantissa fields alone. */
template <class L = L0722>
__device__ __forceinline__ float magnitude(uint64_t w)
{
  return vc::decode_mag<L>(w);
}

/* decode(wa) . decode(wb), taken in spherical form. */
template <class L = L0722, int MODE = PLAIN>
__device__ __forceinline__ float dot(const Params& P, uint64_t wa, uint64_t wb)
{
  return vc::dot_pair<L, MODE>(wa, wb, P);
}

}  // namespace vc_inline
