// CPU emulation build of the device codec (test infrastructure).
//
// Compiles include/vc_device.hpp for the host with libm
// stand-ins for the AMDGPU builtins (v_sin/v_cos/v_rsq/v_rcp are replaced by
// FP64-based equivalents), so the codec's integer logic, octant reduction,
// double-float level arithmetic and exact magnitude path can be checked against
// the oracle on a CPU.  Results differ from the GPU only through those
// transcendental approximations.
#define VC_HOST_EMULATION 1
#include "../../paper_2003_02633_amd/csrc/vc_params.hpp"

using namespace vc;

// as the kernels do: the body under with_compand_mask (compile-time mask and tanh degree when
// both angles are companded)
template <class L, int MODE, int TD>
static void enc_d(const Params& P0, int prec, const float* xyz, uint64_t* out, size_t n)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
    for (size_t i = 0; i < n; i++)
      out[i] = prec == PREC_F64 ? encode_vec<L, MODE, PREC_F64, TD>(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], P)
                                : encode_vec<L, MODE, PREC_F32, TD>(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], P);
  });
}
template <class L, int MODE>
static void enc(const Params& P0, int prec, const float* xyz, uint64_t* out, size_t n)
{
  if (MODE == TANH && tanh_tdeg(P0.wdeg64) == 8) enc_d<L, MODE, 8>(P0, prec, xyz, out, n);
  else enc_d<L, MODE, 15>(P0, prec, xyz, out, n);
}
template <class L, int MODE>
static void dec(const Params& P0, const uint64_t* w, float* out, size_t n)
{
  with_compand_mask<MODE>(P0, [&](const Params& P) {
    for (size_t i = 0; i < n; i++) decode_vec<L, MODE>(w[i], P, out[3 * i], out[3 * i + 1], out[3 * i + 2]);
  });
}

template <class L, int MODE>
static void magc(const Params& P, const uint64_t* w, float* out, size_t n)
{
  for (size_t i = 0; i < n; i++) out[i] = decode_mag_checked<L, MODE>(w[i], P);
}

template <class L, int MODE>
static void dotp(const Params& P, const uint64_t* a, const uint64_t* b, float* out, size_t n)
{
  for (size_t i = 0; i < n; i++) out[i] = dot_pair<L, MODE>(a[i], b[i], P);
}

#define EMU_DISPATCH(R, FN, ...)                      \
  switch ((R).layout * 4 + (R).mode + ((R).mag_round == VC_MAG_TRUNC ? 16 : 0)) { \
    case 0: FN<L0722, PLAIN>(__VA_ARGS__); break;     \
    case 1: FN<L0722, TANH>(__VA_ARGS__); break;      \
    case 2: FN<L0722, COS>(__VA_ARGS__); break;       \
    case 3: FN<L0722, FRAC>(__VA_ARGS__); break;      \
    case 4: FN<L0723, PLAIN>(__VA_ARGS__); break;     \
    case 8: FN<L0823, PLAIN>(__VA_ARGS__); break;     \
    case 12: FN<L1823, PLAIN>(__VA_ARGS__); break;    \
    case 16: FN<L0722T, PLAIN>(__VA_ARGS__); break;   \
    case 17: FN<L0722T, TANH>(__VA_ARGS__); break;    \
    case 18: FN<L0722T, COS>(__VA_ARGS__); break;     \
    case 19: FN<L0722T, FRAC>(__VA_ARGS__); break;    \
    default: return VC_ERROR_UNSUPPORTED_CODEC;       \
  }

extern "C" {

int emu_encode(const vc_codec* c, const float* xyz, uint64_t* out, size_t n)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  if ((st = attach_tables(c, &R)) != VC_SUCCESS) return st;
  EMU_DISPATCH(R, enc, R.P, R.prec, xyz, out, n);
  return 0;
}

int emu_decode(const vc_codec* c, const uint64_t* w, float* out, size_t n)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  EMU_DISPATCH(R, dec, R.P, w, out, n);
  return 0;
}

int emu_magnitude_checked(const vc_codec* c, const uint64_t* w, float* out, size_t n)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  EMU_DISPATCH(R, magc, R.P, w, out, n);
  return 0;
}

int emu_dot_pair(const vc_codec* c, const uint64_t* a, const uint64_t* b, float* out, size_t n)
{
  Resolved R;
  vc_status st = resolve(c, &R);
  if (st != VC_SUCCESS) return st;
  EMU_DISPATCH(R, dotp, R.P, a, b, out, n);
  return 0;
}

int emu_exact_norm(float x, float y, float z, int prec, int keep_sub, uint32_t* j, int* g)
{
  const NormRound nr = exact_norm_round(x, y, z, prec, keep_sub != 0);
  *j = nr.j;
  *g = nr.g;
  return 0;
}

}  // extern "C"
