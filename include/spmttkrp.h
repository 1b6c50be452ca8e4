/*
 * spmttkrp.h -- C ABI of the MI355X (gfx950) sparse MTTKRP library.
 *
 * Sparse MTTKRP over every mode of an N-mode COO tensor inside CP-ALS, with
 * the tensor partitioned per mode by output row (Algorithm 1, Sec. 3.4) and
 * remapped into the next mode's order while each mode is computed (dynamic
 * tensor remapping, Sec. 3.1 and Algorithm 3), so that every output row is
 * accumulated by exactly one workgroup, without global atomics and without
 * intermediate results in HBM (Observations 1 and 2, Sec. 4.3).
 *
 * Conventions for every call:
 *  - Every call returns spt_status; nothing throws across the ABI.  A
 *    failing call leaves a thread-local message in spt_last_error().
 *  - "device" pointers are HIP device allocations of the current device;
 *    "host" pointers are ordinary host memory.  Nothing a caller passes is
 *    kept after the call returns, except the handle the library allocated.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued asynchronously on it unless stated otherwise.
 *  - Indices are 0-based int32, values FP32.  Dimensions and nnz must be
 *    below 2^31; 2 <= nmodes <= 8.  Ranks 8, 16, 32, 64 and 128 are compiled.
 *  - Factor matrices are row-major I_w x R, FP32 or BF16 (spt_dtype).
 *    Factor, output and gradient matrices must start on a 16-byte boundary
 *    (rows are moved as 16-byte vectors); INVALID_ARG otherwise.
 */
#ifndef SPMTTKRP_H
#define SPMTTKRP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spt_status {
    SPT_OK = 0,
    SPT_ERR_INVALID_ARG = 1,   /* NULL where a pointer is required, bad sizes   */
    SPT_ERR_OUT_OF_RANGE = 2,  /* index outside its mode, size beyond int32    */
    SPT_ERR_OOM = 3,           /* host or device allocation failed              */
    SPT_ERR_HIP = 4,           /* a HIP runtime call failed                     */
    SPT_ERR_STATE = 5,         /* tensor not in the order the call requires     */
    SPT_ERR_NOT_SPD = 6,       /* ALS normal matrix not positive definite       */
    SPT_ERR_UNSUPPORTED = 7    /* rank / mode count / layout not compiled       */
} spt_status;

/* Factor storage for the gathers: FP32, or BF16 (the FP32 value rounded to
 * nearest, ties to even; 16-bit patterns).  Accumulation is FP32 either way. */
typedef enum spt_dtype { SPT_F32 = 0, SPT_BF16 = 1 } spt_dtype;

typedef struct spt_tensor_s *spt_tensor_t;  /* opaque, owned by the library */

/* Options of spt_tensor_load_coo; NULL means all defaults. */
typedef struct spt_opts {
    int32_t kappa;      /* partitions per mode (kappa of Alg. 1) = workgroups
                           of each mode's kernel; 0 = default:
                           clamp(ceil(nnz / 2048), 1, 8192)                   */
    int32_t copies;     /* 0 = one tensor copy plus its remapping target
                           (the paper's dynamic remapping); 1 = one
                           mode-ordered copy per mode, no remapping needed  */
    int64_t split_cap;  /* rows with more nonzeros are cut into pieces of at
                           most this many (extension to Alg. 1, see
                           spt_plan_coo); 0 = ceil(nnz / kappa); -1 = never  */
    int32_t prep;       /* where the per-nonzero preprocessing runs: 0 = host
                           threads, 1 = device kernels (row sorts, stream
                           orders, remap ids, packing; Alg. 1's assignment
                           stays on the host).  Same tables and streams
                           either way; ||X||^2 up to FP64 summation order  */
    int32_t dr;         /* how a remapping MTTKRP moves the stream to the next
                           mode's order (Alg. 3), copies == 0 only:
                           0 = a second pass after the elementwise kernel
                           that writes each chunk of consecutive records
                           (the largest power of two of records within
                           2 MB: 131072 records of 12 or 16 bytes; fewer
                           when the tables cannot address that many: see
                           spt_info.remap_chunk) in destination order; the
                           load builds its tables, 6 bytes per nonzero and
                           mode.  1 = fused: the elementwise kernel stores
                           every record at its next position.  The next
                           stream is identical either way                   */
    int32_t layout;     /* record layout of the stream (Sec. 3.5): 0 = chosen
                           by the library (the 12-byte record of layout 4
                           when the indices fit 64 bits; else 32-bit
                           indices for N <= 3; 16-bit fields when every
                           mode has <= 65536 rows; else bit fields of
                           ceil(log2 I_w) bits; else wider records);
                           1 = 32-bit indices (16 / 32 / 48-byte records
                           for N <= 3 / <= 7 / 8); 2 = 16-bit fields
                           (N = 4..6: 16 B, N = 8: 32 B; every mode
                           <= 65536 rows); 3 = packed bit fields (N = 4..6,
                           at most 96 index bits: 16 B); 4 = compact
                           12-byte records, the indices in 64 bits: 32-bit
                           indices for N <= 2, 16-bit fields for N = 4
                           with every mode <= 65536 rows, else packed bit
                           fields when sum_w ceil(log2 I_w) <= 64.  A
                           layout that does not fit fails with
                           SPT_ERR_UNSUPPORTED.  Results are identical for
                           every layout                                     */
    int32_t reserved;   /* must be zero                                      */
} spt_opts;

/* Summary of a loaded tensor (spt_tensor_info). */
typedef struct spt_info {
    int32_t nmodes;
    int32_t cur_mode;        /* mode whose order the stream is in            */
    int32_t kappa;
    int32_t record_bytes;    /* bytes of one packed nonzero record (16/32)   */
    int64_t nnz;
    int64_t dims[8];
    int64_t max_load[8];     /* largest partition of each mode (nonzeros)    */
    int64_t split_rows[8];   /* rows cut into pieces, per mode               */
    double norm_sq;          /* ||X||_F^2 with repeated coordinates summed   */
    double prep_seconds;     /* wall time of the load (preprocessing + upload) */
    int64_t device_bytes;    /* device memory held by the handle             */
    int32_t remap_chunk;     /* records per chunk of the remap pass (each
                                chunk written in destination order); 0 when
                                the handle has no remap pass (opts.dr = 1 or
                                one copy per mode)                           */
} spt_info;

/* mttkrp flags */
#define SPT_FUSE_REMAP_NEXT 1u  /* also scatter the stream into mode (d+1)'s
                                   order (Alg. 3 fused with Alg. 2)           */
#define SPT_AUTO_REMAP 2u       /* remap first if the stream is not in mode d */

/*
 * spt_tensor_load_coo -- preprocess a COO tensor and upload it (Sec. 3.4-3.5,
 * Algorithm 5's input: the tensor ordered by mode 0).
 *   nmodes   number of modes N, 2..8
 *   dims     host int64[N], each in [1, 2^31)
 *   nnz      number of nonzeros, in [0, 2^31)
 *   indices  host int32, mode-major [N][nnz], 0-based
 *   values   host float[nnz]
 *   opts     host, may be NULL
 *   stream   uploads are enqueued on it; the call returns after they finish
 *   out      receives the handle; free it with spt_tensor_free
 * Per mode: degrees, rows ordered by degree, least-filled assignment to
 * kappa partitions, remap ids, then the packed mode-0 stream.  Inputs are
 * copied.  Errors: INVALID_ARG, OUT_OF_RANGE (index outside its mode),
 * UNSUPPORTED (index bits do not fit a 32-byte record), OOM, HIP.
 */
spt_status spt_tensor_load_coo(int32_t nmodes, const int64_t *dims, int64_t nnz,
                               const int32_t *indices, const float *values,
                               const spt_opts *opts, void *stream, spt_tensor_t *out);

/*
 * spt_remap_for_mode -- reorder the stream into `mode`'s order (dynamic
 * remapping, Sec. 3.1) by following each nonzero's remap ids; one pass over
 * the stream (from the current mode to the next with opts.dr == 0: the
 * chunk-ordered remap pass; otherwise a scatter along the chained next
 * positions).  No effect if the stream is already in that order.
 * Errors: INVALID_ARG.
 */
spt_status spt_remap_for_mode(spt_tensor_t t, int32_t mode, void *stream);

/*
 * spt_mttkrp -- spMTTKRP for one output mode (Eq. 1; Algorithms 2-4):
 *   out(i, r) = sum_{nonzeros e with i_mode(e) = i} val(e) *
 *               prod_{w != mode} factors[w](i_w(e), r)
 *   factors  host array of nmodes device pointers, row-major I_w x rank,
 *            element type fdtype; factors[mode] is not read and may be NULL
 *   rank     8, 16, 32, 64 or 128
 *   out      device float, I_mode x rank row-major; OVERWRITTEN (rows with no
 *            nonzero are set to zero)
 *   flags    SPT_FUSE_REMAP_NEXT and/or SPT_AUTO_REMAP
 * The stream must be in `mode`'s order (see spt_tensor_info) unless
 * SPT_AUTO_REMAP is set; otherwise STATE.  With SPT_FUSE_REMAP_NEXT the
 * stream is left in mode (mode+1) mod N's order.  With one copy per mode
 * (opts.copies = 1) any mode may be computed at any time and the flags have
 * no effect.  No global atomics: each output row is written once.
 */
spt_status spt_mttkrp(spt_tensor_t t, int32_t mode, const void *const *factors,
                      spt_dtype fdtype, int32_t rank, float *out, uint32_t flags,
                      void *stream);

/*
 * spt_cp_als_iter -- one CP-ALS sweep over modes 0..N-1 (Sec. 2.1.4;
 * Algorithm 5 extended with the least-squares update of each factor):
 * per mode d, M = mttkrp(d) fused with the remap to d+1; V = Hadamard
 * product of the other factors' Grams (FP64); Y_d = M V^-1 via Cholesky in
 * FP64 (one ridge retry of 1e-12 tr(V)/R, else NOT_SPD); columns of Y_d
 * scaled to unit 2-norm, lambda = the norms.
 *   factors  host array of nmodes device float pointers (FP32 always),
 *            updated in place.  fdtype = SPT_BF16 gathers BF16 copies of them
 *            (kept by the handle, re-rounded after every update); the solve,
 *            Grams and fit use the FP32 factors.
 *   lambda   device double[rank], receives the column norms of the last mode
 *   fit      host double*, receives 1 - ||X - Xhat|| / ||X|| (synchronises
 *            the stream); NULL to skip
 * The stream must be in mode 0's order on entry and is on exit.  With
 * opts.dr = 0 each mode's remap pass runs on a side stream the handle owns
 * (default priority), beside that mode's fixup and factor update; the
 * caller's stream waits for it before the next mode, so all of the call's
 * work is ordered on `stream` as usual.
 * Device workspace is allocated on first use per rank and kept by the
 * handle.  Errors: STATE, UNSUPPORTED, NOT_SPD (reported by the call that
 * synchronises: this one when fit != NULL, else the next), HIP, OOM.
 */
spt_status spt_cp_als_iter(spt_tensor_t t, void *const *factors, spt_dtype fdtype,
                           int32_t rank, double *lambda, double *fit, void *stream);

/*
 * spt_cp_gradient -- loss and gradient of the CP model fitted to the
 * observed nonzeros only (a least-squares fit over the stored entries; the
 * method's spMTTKRP is the adjoint):
 *   m_e  = sum_r prod_w factors[w](i_w(e), r)           (forward, every e)
 *   loss = 1/2 sum_e (x_e - m_e)^2                       (FP64)
 *   grads[d] = dloss/dfactors[d] = MTTKRP of the residuals (m_e - x_e), mode d
 * The forward kernel writes a residual stream (the records with value
 * m_e - x_e); the adjoint is the spMTTKRP kernel over it, remapped mode to
 * mode like the tensor itself.
 *   factors  host array of nmodes device float pointers (I_w x rank)
 *   grads    host array of nmodes device float pointers, overwritten
 *   loss     device double[1], overwritten
 * rank 8, 16, 32 or 64; FP32 factors.  The tensor's stream must be in mode
 * 0's order (it is read, not moved).  The residual streams are allocated on
 * first use and kept by the handle.  Errors: STATE, UNSUPPORTED, HIP, OOM.
 */
spt_status spt_cp_gradient(spt_tensor_t t, const void *const *factors, spt_dtype fdtype,
                           int32_t rank, void *const *grads, double *loss, void *stream);

/*
 * spt_mttkrp_noalloc -- spt_mttkrp for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, flags, results (bit for bit) and errors
 * as spt_mttkrp, and it calls no hipMalloc, hipFree or other allocating
 * routine.  Its only scratch, the partial sums of the mode's split rows
 * (rows whose pieces lie in several partitions), lives in a fixed buffer the
 * library holds on each device for the life of the process: 16 MiB, enough
 * for nslots x rank x 4 bytes (nslots: carry slots of the mode); a larger
 * need returns SPT_ERR_UNSUPPORTED with the size in spt_last_error().  The
 * buffer needs no clearing: every slot a call reads was written earlier in
 * that call.  All calls on one device share it, so calls that overlap on one
 * device (other streams, other threads) race; serialise them.  Hot-row
 * tables are used when an earlier spt_mttkrp call built them for this rank
 * and factor type, else every factor row is read from memory (same results).
 * No kernel timing is recorded.
 */
spt_status spt_mttkrp_noalloc(spt_tensor_t t, int32_t mode, const void *const *factors,
                              spt_dtype fdtype, int32_t rank, float *out, uint32_t flags,
                              void *stream);

/*
 * spt_cp_loss -- the forward half of spt_cp_gradient: m_e at every nonzero,
 * the residual stream (kept by the handle for spt_cp_adjoint) and
 *   loss = 1/2 sum_e (x_e - m_e)^2   (device double[1], overwritten).
 * Arguments, requirements and errors as spt_cp_gradient; no adjoint runs.
 */
spt_status spt_cp_loss(spt_tensor_t t, const void *const *factors, spt_dtype fdtype,
                       int32_t rank, double *loss, void *stream);

/*
 * spt_cp_adjoint -- the backward half of spt_cp_gradient: grads[d] = the
 * MTTKRP of the residual stream of the last spt_cp_loss (or
 * spt_cp_gradient) call on this handle, for every mode d (Eq. (1) with the
 * residuals as values).  `factors` must be the ones that call was given.  The
 * residual stream is left in mode 0's order, so the call may be repeated.
 * Errors: STATE (no residual stream of this rank yet), UNSUPPORTED, HIP, OOM.
 */
spt_status spt_cp_adjoint(spt_tensor_t t, const void *const *factors, spt_dtype fdtype,
                          int32_t rank, void *const *grads, void *stream);

/*
 * spt_copy_probe -- copies `bytes` (a multiple of 16) from device src to
 * device dst with a plain streaming kernel: the copy bandwidth the device
 * reaches, reported beside the HBM peak, and a kernel of known traffic for
 * calibrating memory counters.  Both pointers 16-byte aligned; the ranges
 * must not overlap.  Errors: INVALID_ARG, HIP.
 */
spt_status spt_copy_probe(const void *src, void *dst, int64_t bytes, void *stream);

/* spt_tensor_info -- fills *info (host). */
spt_status spt_tensor_info(spt_tensor_t t, spt_info *info);

/*
 * spt_tensor_get_remap -- remap ids of `mode` as the device holds them:
 * b_host[e] (host int64[nnz]) = position of input nonzero e in mode's
 * stream.  Synchronous.
 */
spt_status spt_tensor_get_remap(spt_tensor_t t, int32_t mode, int64_t *b_host);

/*
 * spt_tensor_get_records -- copies the current stream back and unpacks it:
 * idx_host int32 [N][nnz] and val_host float[nnz] in stream order, plus the
 * mode whose order it is in.  Synchronous.
 */
spt_status spt_tensor_get_records(spt_tensor_t t, int32_t *idx_host, float *val_host,
                                  int32_t *cur_mode);

/* Kernel time of the launches made on one tensor (spt_timing_control). */
typedef struct spt_timing {
    int64_t calls[8];        /* timed spMTTKRP launches per output mode        */
    double ec_ms[8];         /* elementwise kernel (+remap when fused), summed */
    double fixup_ms[8];      /* split-row fixup and empty-row fill, summed     */
    double als_ms[8];        /* CP-ALS dense step after that mode's MTTKRP     */
    double remap_ms[8];      /* staged remap pass (opts.dr == 0), summed;
                                with dr == 1 the remap is inside ec_ms        */
} spt_timing;

/*
 * spt_timing_control -- per-kernel timing with HIP events recorded on the
 * launch stream.  If out != NULL it first waits for the events recorded so
 * far and fills *out (host) with their totals; then enable != 0 clears the
 * totals and starts recording around every later launch on this tensor,
 * enable == 0 stops recording.  Recording adds a few microseconds of host
 * time per launch and nothing to the kernels.
 */
spt_status spt_timing_control(spt_tensor_t t, int32_t enable, spt_timing *out);

/* spt_tensor_free -- releases the handle and its device memory (NULL ok). */
spt_status spt_tensor_free(spt_tensor_t t);

/*
 * spt_plan_coo -- host-only preprocessing, no device needed (for inspection
 * and tests).  Same validation and options as spt_tensor_load_coo.  Outputs
 * (host, caller-allocated, any may be NULL):
 *   part  int32 [N][nnz]   partition of each nonzero in each mode
 *   remap int64 [N][nnz]   remap id b_d(e) = position in mode d's stream
 *   ptr   int64 [N][kappa+1] partition offsets of each stream
 *   kappa_out              the kappa used
 * With part, remap and ptr all NULL only kappa_out is filled (no planning).
 */
spt_status spt_plan_coo(int32_t nmodes, const int64_t *dims, int64_t nnz,
                        const int32_t *indices, const spt_opts *opts, int32_t *part,
                        int64_t *remap, int64_t *ptr, int32_t *kappa_out);

/* Human-readable name of a status. */
const char *spt_status_str(spt_status s);

/* Detail of the last failure on this thread ("" if none). */
const char *spt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMTTKRP_H */
