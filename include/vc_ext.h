/*
 * vc_ext.h -- verification hooks and uncompressed reference kernels of libvc.
 *
 * These are not part of the method; they exist so that its kernels can be
 * verified and measured beside uncompressed storage on the same GPU:
 *   - vcx_axpy_dump runs the same fused axpy kernel as vc_axpy, additionally
 *     writing the single-precision pre-encode sum (for parity checks).
 *   - vcb_* are streaming kernels over uncompressed data: FP32 axpy
 *     (12 bytes per 3-vector), BF16 and FP16 axpy with each 3-vector padded to
 *     four 16-bit values (8 bytes, the same bytes as a code), and a plain copy.
 * Conventions as in vc.h: device pointers owned by the caller, asynchronous on
 * `stream`, synchronous validation, n == 0 is a no-op.
 */
#ifndef VC_EXT_H
#define VC_EXT_H

#include "vc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Same kernel as vc_axpy; also writes c32[i][3] = alpha*decode(a[i]) + decode(b[i]) in float32
 * (the value that was encoded).  c32 is device memory of 3n floats. */
vc_status vcx_axpy_dump(const vc_codec* c, float alpha, const uint64_t* a, const uint64_t* b, uint64_t* out,
                        float* c32, size_t n, hipStream_t stream);

/* c[i] = alpha*a[i] + b[i] over nfloats single-precision values (3 per 3-vector, any
 * arrangement: array-of-structures or structure-of-arrays), one FMA each. */
vc_status vcb_axpy_f32(float alpha, const float* a, const float* b, float* c, size_t nfloats, hipStream_t stream);

/* 3-vectors stored as 4 x bfloat16 (x, y, z, 0): c = alpha*a + b computed in float32 and
 * rounded to nearest-even bfloat16.  a, b, c hold nvec*4 uint16 values (8-byte aligned). */
vc_status vcb_axpy_bf16x4(float alpha, const uint16_t* a, const uint16_t* b, uint16_t* c, size_t nvec,
                          hipStream_t stream);

/* As vcb_axpy_bf16x4 with IEEE binary16 storage. */
vc_status vcb_axpy_f16x4(float alpha, const uint16_t* a, const uint16_t* b, uint16_t* c, size_t nvec,
                         hipStream_t stream);

/* Launch configuration of the streaming compressed axpy (default layout, uniform
 * quantisation) for one encoder precision (VC_PREC_F64 or VC_PREC_F32; -1 sets both):
 * threads per block (128, 256, 512), vectors per thread and grid step (2, 4, or 8 with
 * 256 or 512 threads),
 * non-temporal loads/stores (0/1).  Process-wide; a change may race with launches on other
 * threads (each launch uses the configuration current when it is enqueued).  Unsupported
 * combinations return VC_ERROR_UNSUPPORTED_CODEC and change nothing.
 * vcx_load_tuning reads lines "axpy f64 block=B vpt=V nt=T" (or f32, or no precision for
 * both) from a text file, the cache the autotuner writes; the library applies the file
 * named by $VC_TUNE_CACHE on the first vc_axpy call. */
vc_status vcx_set_stream_config(int precision, int block, int vpt, int nt);
vc_status vcx_get_stream_config(int precision, int* block, int* vpt, int* nt);
vc_status vcx_load_tuning(const char* path);

/* The plan's segments as separate launches (as vc_batch_plan_run_separate), captured once
 * into a second HIP graph on first use and replayed: the launch-overhead baseline between
 * plain separate launches and the persistent kernel. */
vc_status vcx_batch_plan_run_separate_graph(vc_batch_plan* plan, hipStream_t stream);
/* Tile shape of batch plans created from now on for the default codec (other codecs use
 * (2, 4, 8)), in code pairs per lane of a 256-thread workgroup: axpy tiles of 512 ua vectors
 * (ua 1 or 2), dot 512 ud (2, 4 or 8), norm2 512 un (4, 8 or 16); encode tiles are 1024 vectors.
 * Process-wide, chosen by the autotuner (a tuning-cache line "batch ua=A ud=D un=N" applies it);
 * other values return VC_ERROR_UNSUPPORTED_CODEC and change nothing. */
vc_status vcx_set_batch_config(int ua, int ud, int un);
vc_status vcx_get_batch_config(int* ua, int* ud, int* un);
/* Matrix cores of vc_fused_apply, process-wide.  VCX_APPLY_AUTO (the default): the bf16 cores
 * with every FP32 operand split into three bf16 parts and the six part products that keep
 * FP32 accuracy (each term within 3 2^-24 |M_ij| |u_j| before FP32 accumulation), where the
 * operator's three parts fit the LDS beside the output staging (3 rows 32 ceil(cols/32) bf16
 * plus 24 KiB; M of 150 x 125 does), else the FP32 cores; VCX_APPLY_FP32: always the FP32 cores
 * (v_mfma_f32_16x16x4f32).  Results agree to FP32 rounding, not bit for bit.  Other values
 * return VC_ERROR_INVALID_VALUE.  A change may race with launches on other threads. */
enum { VCX_APPLY_AUTO = 0, VCX_APPLY_FP32 = 1 };
vc_status vcx_set_apply_mode(int mode);
int vcx_get_apply_mode(void);
/* Number of tiles the plan's persistent kernel walks and its grid size (workgroups). */
vc_status vcx_batch_plan_info(const vc_batch_plan* plan, uint64_t* total_tiles, uint32_t* grid);

/* Error statistics of the codec over n float32 vectors xyz (device, AoS), the error measures of
 * §2.2-§2.3 evaluated in double precision on the GPU: each finite non-zero vector is encoded by
 * the library's encoder and decoded in FP64 (Eq. (a_inv), (cart2sphere), §2.5 inverse maps);
 *   k = 0: |x_hat - x|/|x|,  k = 1: angle(x, x_hat),  k = 2: |r_hat - |x||/|x|.
 * Vectors that are zero, non-finite, flush to the zero code or saturate are counted in
 * counts[3 (nedges+1)] and left out.  edges: device, nedges ascending FP64 values,
 * 1 <= nedges <= 256; bin = number of edges <= e.  counts: device uint64 [3 (nedges+1) + 1],
 * counts[k (nedges+1) + bin].  stats: device double [9], stats[3k] = sum e, [3k+1] = sum e^2,
 * [3k+2] = max e.  Deterministic; partials are allocated with hipMallocAsync on `stream`. */
vc_status vcx_error_hist(const vc_codec* c, const float* xyz, size_t n, const double* edges, int nedges,
                         uint64_t* counts, double* stats, hipStream_t stream);

/* vc_flux_div_tp on an uncompressed float32 flux F [n_elem][ns][np][3] (the same kernel reading
 * floats): the baseline the compressed flux is compared with. */
vc_status vcb_flux_div_tp_f32(const float* d, int q, int np, const float* F, float* out, size_t n_elem,
                              hipStream_t stream);

/* out[i] = src[idx[i]] for float32 AoS vectors (src [n_src][3]); indices >= n_src give NaN: the
 * uncompressed twin of vc_gather_decode. */
vc_status vcb_gather_f32(const float* src, size_t n_src, const uint32_t* idx, size_t n, float* out,
                         hipStream_t stream);

/* dst[0:bytes) = src[0:bytes): the attainable-bandwidth reference.  16-byte aligned. */
vc_status vcb_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

/* The codec's resolved constants for the device functions of vc_inline.hpp (the inline use of
 * the method: encode and decode inside the caller's own kernels, §1 and Alg. fr_fdiv_comp).
 * Writes `size` bytes of the constants block to params (host memory, owned by the caller), which
 * a kernel takes by value as vc_inline::Params; size must equal vcx_inline_params_size().
 * Returns VC_ERROR_INVALID_VALUE for a NULL pointer or a wrong size, and the codec's own
 * validation errors (VC_ERROR_UNSUPPORTED_CODEC) otherwise.  The kernel must instantiate the
 * device functions for the codec's layout, mode and encoder precision. */
vc_status vcx_inline_params(const vc_codec* c, void* params, size_t size);
size_t vcx_inline_params_size(void);

#ifdef __cplusplus
}
#endif
#endif /* VC_EXT_H */
