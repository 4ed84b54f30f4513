/*
 * fzo.h -- interface of the ORACLE (test infrastructure only; see fzo.c).
 * Not included by, and sharing nothing with, the HIP library.
 */
#ifndef FZO_H
#define FZO_H
#include <stdint.h>

#define FZO_EB_ABS 0
#define FZO_EB_REL 1
#define FZO_EB_PWREL 2

/* data-dependent error bits (OR-ed into the stream header status word) */
#define FZO_ERR_NONFINITE 1u
#define FZO_ERR_EB_RANGE 2u
#define FZO_ERR_OUTLIER_CAP 4u

/* decompressor return codes */
#define FZO_DERR_ARG 1
#define FZO_DERR_STREAM 2
#define FZO_DERR_VERSION 3
#define FZO_DERR_STATUS 4

int64_t fzo_bound(int rank, const int64_t *dims);
int64_t fzo_header_bytes(int rank, const int64_t *dims);
int64_t fzo_n_chunks(int rank, const int64_t *dims);
int fzo_eb_params(const float *x, int64_t n, double eb, int eb_mode, float *ebx2, float *inv, float *vmin,
                  float *vmax);
int fzo_prequant(const float *x, int64_t n, float inv, int32_t *q);
int fzo_prequant_pw(const float *x, int64_t n, uint32_t step, int32_t *q);
float fzo_dequant_pw(int32_t q, uint32_t step);
int fzo_code_of(int32_t d, uint16_t *code);
int32_t fzo_delta_of(uint16_t code);
int fzo_lorenzo_field(const int32_t *q, int rank, const int64_t *dims, int32_t *delta);
int64_t fzo_chunk_codes(const float *x, int rank, const int64_t *dims, float inv, int64_t c, uint16_t *codes_out);
int64_t fzo_compress(const float *x, int rank, const int64_t *dims, double eb, int eb_mode, uint8_t *out,
                     int64_t cap, uint32_t *status_out, int threads);
int fzo_decompress(const uint8_t *s, int64_t size, float *x, int rank, const int64_t *dims);
/* the same with the chunks spread over `threads` OpenMP threads (0: default) */
int fzo_decompress_threads(const uint8_t *s, int64_t size, float *x, int rank, const int64_t *dims, int threads);
/* global = 1: the field-global Lorenzo predictor (header byte 15); fzo_decompress reads either */
int64_t fzo_compress_pred(const float *x, int rank, const int64_t *dims, double eb, int eb_mode, int global,
                          uint8_t *out, int64_t cap, uint32_t *status_out, int threads);
/* fp64 input (ABS and REL modes) */
int fzo_eb_params_f64(const double *x, int64_t n, double eb, int eb_mode, double *ebx2, double *inv,
                      double *vmin, double *vmax);
int fzo_prequant_f64(const double *x, int64_t n, double inv, int32_t *q);
int64_t fzo_compress_f64(const double *x, int rank, const int64_t *dims, double eb, int eb_mode,
                         uint8_t *out, int64_t cap, uint32_t *status_out, int threads);
int fzo_decompress_f64(const uint8_t *s, int64_t size, double *x, int rank, const int64_t *dims);
#endif
