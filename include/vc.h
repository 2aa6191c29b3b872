/*
 * vc.h -- C ABI of libvc, the MI355X (gfx950) implementation of the inline
 * 3-vector compression of Trojak & Witherden, "Inline Vector Compression for
 * Computational Physics" (arXiv 2003.02633).
 *
 * A single-precision 3-vector (96 bits) is stored as one 64-bit code: two
 * quantised spherical angles plus a shortened floating-point magnitude
 * (§2.1-2.3; default layout <0,7,22>-17-18, Fig. comp_regimes c).  Encode and
 * decode run inside streaming kernels; the paper's benchmark operation is the
 * compressed vector addition of §5, exposed here as an axpy.
 *
 * Conventions for every entry point
 *   - Pointers named d_* or documented as "device" are device (HBM) pointers
 *     owned by the caller; the library never frees them.  Host pointers are
 *     documented as such.
 *   - Validation is synchronous: on any error the call returns a status and
 *     enqueues nothing.  Kernel launches are asynchronous on `stream`
 *     (NULL = the null stream); a launch failure returns VC_ERROR_LAUNCH.
 *     Faults inside a kernel surface at the caller's next stream sync.
 *   - n == 0 is a successful no-op; NULL data pointers are allowed then.
 *   - Codes are uint64 (8-byte aligned).  Cartesian vectors are float32,
 *     array-of-structures [n][3] (4-byte aligned; 16-byte alignment takes the
 *     fast path).
 *   - Non-finite input vectors encode to the reserved code (exponent field
 *     all ones, other fields zero), which decodes to NaN.
 *   - The library never synchronises the device implicitly, except where
 *     documented (plan creation).
 *
 * Environment
 *   VC_TUNE_CACHE  file of axpy launch configurations, applied on the first
 *                  vc_axpy call (format in vc_ext.h, vcx_load_tuning).
 *   VC_LOG         set to a non-empty value other than "0": vc_encode,
 *                  vc_decode, vc_axpy, vcx_axpy_dump, vc_dot and vc_norm2 each
 *                  write one line to stderr when they return (codec fields, n,
 *                  the axpy launch configuration, the status).
 */
#ifndef VC_H
#define VC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VC_ABI_VERSION 1

typedef enum {
  VC_SUCCESS = 0,
  VC_ERROR_INVALID_VALUE = 1,     /* NULL pointer with n > 0, bad size or option */
  VC_ERROR_MISALIGNED = 2,        /* code pointer not 8-byte aligned, float pointer not 4-byte aligned */
  VC_ERROR_UNSUPPORTED_CODEC = 3, /* layout/mode combination not built into the library */
  VC_ERROR_LAUNCH = 4,            /* kernel launch failed (hipGetLastError) */
  VC_ERROR_HIP = 5,               /* another HIP runtime call failed */
  VC_ERROR_OUT_OF_MEMORY = 6,     /* library-owned allocation failed */
  VC_ERROR_OVERLAP = 7            /* output partially overlaps an input */
} vc_status;

/* bit layouts <s,e,m>-p-t of §2.2-2.3 (fields MSB->LSB: sign, exponent, mantissa, n_phi, n_theta) */
typedef enum {
  VC_LAYOUT_0_7_22_17_18 = 0, /* default, Fig. comp_regimes c, exponent bias 80 */
  VC_LAYOUT_0_7_23_17_17 = 1, /* Fig. comp_regimes b, bias 80 */
  VC_LAYOUT_0_8_23_16_17 = 2, /* Fig. comp_regimes a, IEEE exponent, bias 127 */
  VC_LAYOUT_1_8_23_16_16 = 3  /* base scheme of §2.2: plain float32 magnitude bits above n_phi, n_theta */
} vc_layout;

/* angle discretisation: uniform (Eq. a_disc), companding maps (§2.5), fractional split (§2.4) */
typedef enum { VC_MODE_PLAIN = 0, VC_MODE_TANH = 1, VC_MODE_COS = 2, VC_MODE_FRACSPLIT = 3 } vc_mode;

/* magnitude rounding: nearest-even of the exact norm (default), or the paper-literal
 * truncation of the single-precision magnitude's trailing mantissa bits (§2.3): the norm
 * rounded to nearest-even at 24 bits, then its low 23 - m mantissa bits dropped.  With a
 * 23-bit mantissa nothing is dropped and the two give the same codes.  Decoding does not
 * depend on it. */
typedef enum { VC_MAG_RNE = 0, VC_MAG_TRUNC = 1 } vc_mag_round;

enum { VC_COMPAND_PHI = 1, VC_COMPAND_THETA = 2 };

/* arithmetic of the encoder's norm, angle ratios and level coordinates: double precision
 * (the paper's implementation section prescribes it for phi; full-rate FMA on MI355X), or
 * single precision only, with double-float error-free transformations.  Both produce the
 * same codes up to the one-ulp window; decode and all post-decode arithmetic are single
 * precision in both.  The companding modes (tanh, cosine) need VC_PREC_F64; with VC_PREC_F32
 * every entry point returns VC_ERROR_UNSUPPORTED_CODEC for them. */
typedef enum { VC_PREC_F64 = 0, VC_PREC_F32 = 1 } vc_precision;

/* Codec description.  Plain data, owned by the caller; build it with vc_codec_init
 * and adjust fields before use.  struct_size versions the layout. */
typedef struct {
  uint32_t struct_size;   /* = sizeof(vc_codec) */
  uint32_t layout;        /* vc_layout */
  uint32_t mode;          /* vc_mode */
  uint32_t mag_round;     /* vc_mag_round */
  uint32_t compand_mask;  /* VC_COMPAND_* bits: angles a companding map applies to */
  float gamma;            /* tanh companding parameter (§2.5), in (0, 1] */
  uint64_t frac_P;        /* fractional split: n_phi_max + 1 (§2.4, Eq. q_split) */
  uint32_t precision;     /* vc_precision of the encoder */
  uint32_t reserved0;     /* must be 0 */
} vc_codec;

/* Fill *c with the plain codec of `layout` ("0,7,22-17-18", "0,7,23-17-17",
 * "0,8,23-16-17", "1,8,23-16-16"; NULL selects the default <0,7,22>-17-18),
 * RNE magnitude, companding of both angles with gamma = 0.5 when a companding mode
 * is later selected, frac_P = 2^17, double-precision encoder arithmetic.  Host-only. */
vc_status vc_codec_init(vc_codec* c, const char* layout);

/* Encode n float32 vectors (device, AoS [n][3]) into n codes (device).  §3: three
 * single-precision numbers in, 64 bits out; angles by Eq. (a_disc) (round half up),
 * magnitude by §2.3.  `xyz` and `codes` must not overlap. */
vc_status vc_encode(const vc_codec* c, const float* xyz, uint64_t* codes, size_t n, hipStream_t stream);

/* Decode n codes (device) into float32 vectors (device, AoS [n][3]): Eq. (a_inv) and
 * Eq. (cart2sphere).  The zero code decodes to (0,0,0), the reserved code to NaN. */
vc_status vc_decode(const vc_codec* c, const uint64_t* codes, float* xyz, size_t n, hipStream_t stream);

/* Compressed axpy, the vector-addition kernel of §5 with a scale: for each i,
 * c[i] = encode(alpha * decode(a[i]) + decode(b[i])), one single-precision fused
 * multiply-add per component.  a, b, c are device code arrays of length n; c may
 * alias a or b exactly (in-place), partial overlap returns VC_ERROR_OVERLAP. */
vc_status vc_axpy(const vc_codec* c, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* out,
                  size_t n, hipStream_t stream);

/* d_out[0] = sum_i decode(a[i]) . decode(b[i]), single-precision products with
 * single-precision accumulation (fixed reduction order, deterministic).  d_out is
 * one device float.  The paper defines no dot product of its own: this is the plain sum
 * of products of the vectors that Eq. (a_inv) and Eq. (cart2sphere) decode.  The per-block
 * partials go to a stream-ordered allocation (hipMallocAsync) freed before return. */
vc_status vc_dot(const vc_codec* c, const uint64_t* a, const uint64_t* b, size_t n, float* d_out,
                 hipStream_t stream);

/* vc_dot without allocation, for callers that cannot call hipMalloc (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same kernels and the same
 * result, bit for bit, as vc_dot, with the per-block partial sums in a library-owned device array
 * of 2048 floats (8 KiB) instead of a hipMallocAsync buffer.  Every n fits (the partials never
 * exceed 2048); a larger partial count would return VC_ERROR_INVALID_VALUE.  The array is
 * allocated with the code object, one per device, and held until the process ends; its address
 * is looked up on the first call on a device (the device current at the call; the stream must
 * belong to it).  Calls that overlap on one device (two streams, or two host threads) share the
 * array and race: serialise them.  Each call writes every partial it reads, so nothing needs
 * clearing between calls. */
vc_status vc_dot_noalloc(const vc_codec* c, const uint64_t* a, const uint64_t* b, size_t n, float* d_out,
                         hipStream_t stream);

/* d_out[0] = sum_i |decode(a[i])|^2, from the magnitude field alone (|x_hat| equals the
 * stored magnitude exactly in real arithmetic), single-precision accumulation.  Like vc_dot,
 * not a paper operation: the plain sum of squared magnitudes of the vectors of §2.3. */
vc_status vc_norm2(const vc_codec* c, const uint64_t* a, size_t n, float* d_out, hipStream_t stream);

/* Fused decode + dense apply, the operator pattern of Alg. (fr_fdiv_comp): for each
 * element e, out[e] (rows x 3, float32) = M (rows x cols, float32 row-major, device)
 * times decode(U[e]) (cols vectors, codes [n_elem][cols], device).  Contraction on
 * the matrix cores in single precision with single-precision accumulation.
 * 1 <= rows <= 256, 1 <= cols <= 256 and 4 ceil(cols/4) RS <= 20480, RS = rows rounded up to
 * 24 mod 32 (the operator is staged in LDS with row stride RS), else VC_ERROR_INVALID_VALUE. */
vc_status vc_fused_apply(const vc_codec* c, const float* M, int rows, int cols, const uint64_t* U,
                         float* out, size_t n_elem, hipStream_t stream);

/* Divergence of a compressed flux on hexahedral flux-reconstruction elements, Alg. (fr_fdiv_comp)
 * of §4 (step 10 of the FR right-hand side): for element i, solution point k and equation p,
 *   out[i][k][p] = sum_j sum_c D[c ns + j][k] decode(F[i][j][p])[c],
 * with the tensor-product divergence operator of q = p_FR + 1 Gauss-Legendre points per
 * direction, ns = q^3, point index j = jx + q jy + q^2 jz, given by its 1D factors:
 * D[c ns + j][k] = d[c][j_c][k_c] when the two other coordinates of j and k agree, else 0.
 *   d   : device float32 [3][q][q], d[c][a][b] = derivative in direction c of the basis
 *         polynomial of node a, at node b (element scaling included);
 *   F   : device codes [n_elem][ns][np], one row of the np x 3 flux tensor per code (Eq. eulerF);
 *   out : device float32 [n_elem][ns][np], must not overlap F.
 * 2 <= q <= 6, 1 <= np <= 8.  Single-precision decode and accumulation. */
vc_status vc_flux_div_tp(const vc_codec* c, const float* d, int q, int np, const uint64_t* F, float* out,
                         size_t n_elem, hipStream_t stream);

/* Random access to compressed vectors (fixed-rate codes are individually addressable, §1; the
 * interface steps of flux reconstruction read neighbours' values through a connectivity array,
 * Table fr_nse steps 2 and 8).
 * vc_gather_decode : out[i] = decode(codes[idx[i]]) for i < n; codes has n_src entries, idx
 *   (device uint32 [n]) entries >= n_src are not dereferenced and give (NaN, NaN, NaN); out is
 *   float32 AoS [n][3] and must not overlap codes or idx.
 * vc_scatter_encode: codes[idx[i]] = encode(xyz[i]) for i < n; idx entries >= n_dst are
 *   skipped; with repeated indices the code written is one of the candidates, unspecified which.
 * Single-precision decode; the encoder of the codec's precision. */
vc_status vc_gather_decode(const vc_codec* c, const uint64_t* codes, size_t n_src, const uint32_t* idx, size_t n,
                           float* out, hipStream_t stream);
vc_status vc_scatter_encode(const vc_codec* c, const float* xyz, const uint32_t* idx, size_t n, uint64_t* codes,
                            size_t n_dst, hipStream_t stream);

/* ---- batched persistent launch over a segment table ---- */
typedef enum { VC_OP_AXPY = 0, VC_OP_DOT = 1, VC_OP_NORM2 = 2, VC_OP_ENCODE = 3 } vc_op;

/* One segment.  AXPY: out[i] = encode(alpha decode(a[i]) + decode(b[i])), codes.
 * DOT: *(float*)out = a . b.  NORM2: *(float*)out = |a|^2.  ENCODE: a = float AoS
 * vectors, out = codes.  All pointers are device pointers. */
typedef struct {
  uint32_t op;      /* vc_op */
  float alpha;
  uint64_t n;
  const void* a;
  const void* b;
  void* out;
} vc_segment;

typedef struct vc_batch_plan vc_batch_plan;

/* Build a plan for `nseg` segments (host array, copied; 0 <= nseg <= 2^20).  Each segment is
 * cut into tiles (512 to 4096 vectors, by operation and the tuned tile shape); one persistent
 * kernel walks all tiles of all segments with a static grid stride, and a second kernel sums
 * the per-wave partials of each dot/norm2 segment in a fixed order (deterministic; an empty
 * reduction segment yields 0).  Both are
 * captured into a HIP graph.  Segments run concurrently, so no segment may write memory that
 * another segment reads or writes (VC_ERROR_OVERLAP); within a segment the rules of the
 * single-call entry points hold (axpy may run in place).  Pointer and size checks as for
 * those entry points.  Allocates the device segment table and partial-sum scratch and
 * synchronises `stream` once; the plan owns them until vc_batch_plan_destroy.  Segment data
 * pointers are stored, not copied: they must stay valid while the plan is run. */
vc_status vc_batch_plan_create(vc_batch_plan** plan, const vc_codec* c, const vc_segment* segs, int nseg,
                               hipStream_t stream);
/* Replay the plan's graph on `stream` (asynchronous).  Runs on one stream at a time. */
vc_status vc_batch_plan_run(vc_batch_plan* plan, hipStream_t stream);
/* Run the same segments as separate kernel launches, one per segment (the baseline
 * the persistent launch is compared with). */
vc_status vc_batch_plan_run_separate(vc_batch_plan* plan, hipStream_t stream);
/* Free the plan; no run of it may still be in flight. */
vc_status vc_batch_plan_destroy(vc_batch_plan* plan);

/* Human-readable name of a status.  Static string, never NULL. */
const char* vc_status_string(vc_status s);
/* Library version string, static. */
const char* vc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VC_H */
