/*
 * det.h -- exact integer determinant on one MI355X (gfx950).
 *
 * The data-parallel hot path of Dumas and Urbanska's introspective integer
 * determinant ("An introspective algorithm for the integer determinant"):
 * LU modulo word-size primes over a batch of primes (the Chinese-remaindering
 * side, Section 2.1 and Alg. 2.1) and Dixon p-adic lifting with A^{-1} mod p
 * (the LargestInvariantFactor side, Section 2.2), combined on the host as in
 * Section 4 (Alg. 4.1 with one solving: det = s~_n * (det / s~_n)).
 *
 * Conventions for every entry point:
 *  - Return value: det_status, DET_OK (0) on success.  No C++ exception and
 *    no longjmp crosses this boundary.  On failure the outputs are left in an
 *    unspecified state and det_last_error(ctx) describes the cause.
 *  - Matrices: row-major n x n int64 with leading dimension lda >= n (in
 *    elements).  The pointer may be host or device memory; the library asks
 *    the HIP runtime which one it is.  Entries must satisfy |a_ij| < 2^31.
 *  - Ownership: the caller owns every input and output buffer.  The library
 *    keeps no caller pointer after a call returns and allocates device memory
 *    only inside the context (freed by det_ctx_destroy).
 *  - Calls are synchronous with respect to the host: they return after the
 *    work queued on the context's stream has finished.  A context must not be
 *    used from two threads at the same time.
 *  - n = 0 is accepted: the determinant of the empty matrix is 1.
 */
#ifndef PAPER_CS_0511066_AMD_DET_H
#define PAPER_CS_0511066_AMD_DET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DET_OK = 0,
  DET_E_INVALID = 1,          /* bad argument: null pointer, n < 0, lda < n, k < 0 ... */
  DET_E_NOT_PRIME = 2,        /* a modulus is not an odd prime */
  DET_E_PRIME_RANGE = 3,      /* modulus outside the range the chosen path supports */
  DET_E_SINGULAR_MOD_P = 4,   /* dixon_lift: p divides det(A) */
  DET_E_OVERFLOW = 5,         /* an entry has |a_ij| >= 2^31, or a bound would overflow */
  DET_E_NOMEM = 6,            /* device or host allocation failed */
  DET_E_BUFFER_TOO_SMALL = 7, /* det_introspective: limb_cap too small (see limb_count) */
  DET_E_DEVICE = 8            /* a HIP runtime call failed */
} det_status;

typedef enum {
  DET_PATH_AUTO = 0,          /* library choice (int8 limbs when every prime allows it) */
  DET_PATH_FP64 = 1,          /* trailing updates on FP64 MFMA, primes < 2^26 */
  DET_PATH_INT8 = 2           /* trailing updates on int8 MFMA with 3 signed limbs, primes < 2^23 */
} det_path;

typedef struct det_ctx det_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * workspace the context may hold (0 = no cap).  The context owns a HIP
 * stream of default priority.  Returns DET_E_DEVICE if the device cannot be
 * used. */
det_status det_ctx_create(int device, size_t hbm_budget_bytes, det_ctx **out);

/* Free everything the context allocated.  NULL is ignored. */
void det_ctx_destroy(det_ctx *ctx);

/* Run subsequent work on `hip_stream` (a hipStream_t, borrowed: the library
 * never destroys it).  NULL restores the context's own stream. */
det_status det_ctx_set_stream(det_ctx *ctx, void *hip_stream);

/* Human-readable name of a status code (static storage). */
const char *det_status_str(det_status s);

/* Message describing the last failure on this context (owned by ctx). */
const char *det_last_error(const det_ctx *ctx);

/*
 * CRA side (Section 2.1: each modular determinant comes from an LU
 * factorisation modulo p_i; Alg. 2.1 computes det(A) mod p_i for each drawn
 * prime).
 *
 * residues[j] = det(A) mod primes[j], canonical in [0, primes[j]).  A
 * residue 0 is a valid result (p_j divides det(A), or A is singular), not an
 * error.  primes: host array of nprimes odd primes, each < 2^26 for
 * DET_PATH_FP64 and < 2^23 for DET_PATH_INT8 (else DET_E_PRIME_RANGE);
 * residues: host array of nprimes entries.  Every prime is checked with a
 * deterministic primality test (DET_E_NOT_PRIME).
 */
det_status det_mod_primes(det_ctx *ctx, const int64_t *A, int64_t n, int64_t lda,
                          const uint32_t *primes, int64_t nprimes, uint32_t *residues,
                          det_path path);

/*
 * det_mod_primes without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same result as det_mod_primes(..., DET_PATH_FP64), from the
 * same kernels, but every device buffer comes from one static 64 MiB array
 * per device that the library holds until the process ends; no context is
 * used and nothing is allocated.
 *   device      HIP device to run on (made current for the call, then the
 *               caller's current device is restored).
 *   hip_stream  hipStream_t on that device (NULL: its null stream), borrowed.
 *   A           DEVICE pointer, row-major n x n int64, leading dimension lda,
 *               |a_ij| < 2^31 (checked: DET_E_OVERFLOW).
 *   primes      host array of nprimes odd primes < 2^26.
 *   residues    host array of nprimes outputs, det(A) mod primes[j].
 * Returns DET_E_INVALID when A is not device memory or when the workspace of
 * one prime at this n does not fit the array (n above about 4000); primes are
 * processed in batches that fit.  The array keeps the last call's contents;
 * calls that overlap on one device (other threads, other streams) race on it.
 * The call returns after its work on hip_stream has finished.
 */
det_status det_mod_primes_noalloc(int device, void *hip_stream, const int64_t *A, int64_t n,
                                  int64_t lda, const uint32_t *primes, int64_t nprimes,
                                  uint32_t *residues);

/*
 * LIF side (Section 2.2: LargestInvariantFactor solves A x = b by Dixon
 * p-adic lifting).  With r_0 = b:
 *     x_i = A^{-1} r_i mod p  in [0, p)^n,     r_{i+1} = (r_i - A x_i) / p,
 * so that sum_{i<k} x_i p^i = A^{-1} b (mod p^k).
 * digits[i*n + j] = x_i[j] for 0 <= i < k, 0 <= j < n (host array, k*n
 * entries).  b: host array of n int64 with |b_j| < 2^62 / (n + 1).
 * p: odd prime with 2^8 < p < 2^26.  Returns DET_E_SINGULAR_MOD_P when p
 * divides det(A).  A device pointer for A is used in place.
 */
det_status dixon_lift(det_ctx *ctx, const int64_t *A, int64_t n, int64_t lda, const int64_t *b,
                      uint32_t p, int64_t k, uint32_t *digits);

/*
 * Dixon lifting of m right-hand sides at once (the system A X = B with
 * several right-hand sides, Section 3.2: the lifting step becomes a product
 * with an n x m matrix):  digits[(h*k + i)*n + j] = x_{h,i}[j], the i-th
 * base-p digit of A^{-1} b_h, for h < m, i < k, j < n -- exactly what
 * dixon_lift returns for b_h alone.  B: host array, n x m int64 row-major
 * (B[j*m + h]), each |B_jh| < 2^62 / (n + 1); digits: host array of m*k*n
 * entries, owned by the caller.  In the FP64 three-digit form two right-hand
 * sides share one launch (the planes of A^{-1}, the rows of A and every
 * exchange between workgroups); other forms lift them one after the other.
 * Errors as dixon_lift; m = 0 returns DET_OK.
 */
det_status dixon_lift_multi(det_ctx *ctx, const int64_t *A, int64_t n, int64_t lda,
                            const int64_t *B, int64_t m, uint32_t p, int64_t k, uint32_t *digits);

/*
 * Several Dixon liftings side by side (Section 6: p-adic liftings with
 * different primes in parallel, each with fewer iterations; their results
 * meet by Chinese remaindering, as det_introspective does):
 * digits[(z*k + i)*n + j] = x_i[j], the i-th base-p_z digit of A^{-1} b,
 * for each of the np distinct primes p_z -- exactly what dixon_lift returns
 * for p_z alone.  1 <= np <= 4; primes: host array; digits: host array of
 * np*k*n entries, owned by the caller.  When the FP64 three-digit form
 * applies to every prime (p_z < 2^25, n ||A|| p_z < 2^53, n <= 1024) and np
 * of its grids fit on the device, the inverses come from one batched LU and
 * the liftings share one launch (each prime its own workgroups); otherwise
 * the primes are lifted one after the other.  Errors as dixon_lift, plus
 * DET_E_INVALID for repeated primes.
 */
det_status dixon_lift_primes(det_ctx *ctx, const int64_t *A, int64_t n, int64_t lda,
                             const int64_t *b, const uint32_t *primes, int64_t np, int64_t k,
                             uint32_t *digits);

typedef struct {
  double log2_inv_eps;   /* early termination: failure probability < 2^-log2_inv_eps (default 64) */
  int certify;           /* 1: ignore early termination; reconstruct det/s_n up to the Hadamard bound */
  uint64_t seed;         /* seed for the prime draws and the right-hand sides */
  int n_rhs;             /* i_max, the most Dixon solvings (Alg. 4.1), default 1, at most 8.  All
                            solvings share one prime and one inverse; from the second on, the
                            extended bonus (Section 3.2) turns i solutions into
                            pi~_i = s~^i / gcd(det(R N), s~^i), a factor of s_n ... s_{n-i+1},
                            and K = lcm of everything found */
  int prime_bits;        /* CRA primes are drawn from (2^(b-1), 2^b); default 23 (max 23 for int8, 26 for fp64) */
  det_path path;         /* trailing-update path of the CRA loop */
  int adaptive;          /* 1 (default): Alg. 4.1's loop -- after each solving the CRA on det/K
                            resumes for at most that solving's time and returns on early
                            termination; from the second solving on, the loop turns to the CRA
                            when pi~_i = pi~_{i-1} or, by Section 5.3's rule, when
                            log2(pi~_i / pi~_{i-1}) <= (time(solving) / time(LU)) log2(l).
                            0: exactly n_rhs solvings, then the CRA on det/K */
  int lift_primes;       /* liftings side by side (Section 6: several p-adic liftings in
                            parallel, each with fewer steps, combined by Chinese remaindering):
                            0 (default) picks the number, 1 .. 4 asks for at most that many.
                            Applies to the three-digit lifting (n <= 1024); each solving then
                            lifts modulo every one of the primes, to k digits each with
                            prod p_z^k above the reconstruction bound */
} det_opts;

typedef struct {
  int64_t primes_used;     /* CRA primes whose residues entered the reconstruction */
  int64_t lifting_steps;   /* Dixon steps over all solvings */
  int64_t sn_bits;         /* bit length of the divisor K of det(A) found by the solvings */
  int64_t et_rounds;       /* batches of CRA primes launched */
  int64_t hadamard_bits;   /* log2 of the Hadamard bound used */
  int early_terminated;    /* 1 if the CRA stopped by early termination */
  int bonus_factors;       /* i when the extended bonus pi~ (i solvings) entered the divisor;
                              -i when a rational reconstruction of the bonus failed (only the
                              denominators found entered it); 0 when the bonus did not run */
  double t_lif_ms;         /* device + host time of the solvings */
  double t_cra_ms;         /* time of the modular determinants */
  double t_host_ms;        /* time of reconstruction on the host */
  int64_t solvings;        /* Dixon solvings done (Alg. 4.1's i) */
  int timing_switch;       /* 1 when Section 5.3's time rule ended the solvings */
  double t_solve_ms;       /* time of the last solving (lifting + reconstruction) */
  double t_lu_ms;          /* measured device time per modular determinant (batched) */
  int64_t lift_primes;     /* primes lifted side by side in each solving */
} det_report;

/* Fill *opts with the defaults above. */
void det_opts_default(det_opts *opts);

/*
 * Exact det(A) by the introspective scheme of Section 4 (Alg. 4.1 with
 * i_max = opts->n_rhs, default 1): s~_n from Dixon lifting and rational
 * reconstruction (and, from the second solving on, the extended bonus), then
 * the early-terminated CRA loop (Alg. 2.1) on det(A)/K, and
 * det = K * (det/K).  See det_opts.adaptive for the loop's stopping rules.
 * Output: *sign in {-1, 0, +1}; |det| as little-endian base-2^32 limbs in
 * mag[0 .. *limb_count).  If limb_cap is too small the call returns
 * DET_E_BUFFER_TOO_SMALL with *limb_count = limbs needed (call again).
 * opts and report may be NULL.  With certify = 0 the result is correct with
 * probability >= 1 - 2^-log2_inv_eps (Lemma 2.1(iv)); with certify = 1 it is
 * always correct.
 */
det_status det_introspective(det_ctx *ctx, const int64_t *A, int64_t n, int64_t lda,
                             const det_opts *opts, int *sign, uint32_t *mag, int64_t limb_cap,
                             int64_t *limb_count, det_report *report);

/*
 * Many exact determinants in one call (the batched workload): a set of
 * independent dense matrices of any orders.  Each matrix follows the
 * early-terminated Chinese remaindering of Section 2.1 (Alg. 2.1, run length
 * of Lemma 2.1(iv); certify = 1: up to the Hadamard bound) with its own primes,
 * drawn from the stream seeded by opts->seed + i, so its result does not
 * depend on the rest of the batch.  The rounds of all matrices run together:
 * every (matrix, prime) LU item of order <= 512 of a round is one entry of a
 * device work queue, sorted by decreasing order and run by one persistent
 * launch (HIP graph: queue reset, launch and copies), in the launch shape
 * that det_autotune chose for the orders present; larger matrices take the
 * blocked batched LU of det_mod_primes beside it.  Section 6 observes that
 * the LU runs of one CRA step are independent; so are those of different
 * matrices.
 *   A[i]        row-major n[i] x n[i] int64, leading dimension lda[i], host or
 *               device pointer, owned by the caller and only read; |a| < 2^31.
 *   opts        NULL = defaults; log2_inv_eps, certify, seed and prime_bits are
 *               used (path applies to the matrices above 512).
 *   sign[i]     -1, 0 or +1.
 *   mag         count x limb_stride uint32: |det A[i]| as little-endian limbs
 *               from mag + i * limb_stride; limb_count[i] limbs are used.
 *   status[i]   per-matrix status; DET_E_BUFFER_TOO_SMALL with the needed
 *               limb count in limb_count[i] when limb_stride is too small.
 *   t_done_ms   optional: time at which matrix i's result was ready, in ms
 *               since the call started.
 * The first call on a context without a launch-shape table runs det_autotune
 * (with the cache file named by the environment variable DET_AUTOTUNE_CACHE,
 * if set).  Returns DET_OK when every matrix succeeded, else the status of the
 * first failing matrix (see det_last_error).
 */
det_status det_batch(det_ctx *ctx, int64_t count, const int64_t *const *A, const int64_t *n,
                     const int64_t *lda, const det_opts *opts, int *sign, uint32_t *mag,
                     int64_t limb_stride, int64_t *limb_count, det_status *status,
                     double *t_done_ms);

/*
 * Autotuner of the persistent LU kernel: for each order bucket (<= 64, 128,
 * 256, 512) it times every launch shape (panel width 32 with one workgroup per
 * CU, panel width 16 with one, or two with registers capped) on a seeded batch
 * of 4 items per CU, checks that all shapes give the same residues, and keeps
 * the fastest.
 * cache_path (may be NULL): a JSON file read instead of measuring when it
 * matches this device (architecture name and CU count), and written after
 * measuring.
 */
det_status det_autotune(det_ctx *ctx, const char *cache_path);

/* The context's launch-shape table: up to cap entries (bucket order limit,
 * kernel variant 1 = panel width 32, 2 = width 16, 3 = width 16 two per CU;
 * workgroups per CU; measured items per ms); *count = number of entries. */
det_status det_autotune_read(const det_ctx *ctx, int64_t cap, int32_t *nmax, int32_t *variant,
                             int32_t *blocks_per_cu, double *items_per_ms, int64_t *count);

/*
 * Serving: a stream of determinant requests on one context, admitted by HBM
 * footprint and served with continuous batching.  An engine thread owns the
 * context from det_server_create to det_server_destroy (the caller must not
 * use ctx meanwhile, and must destroy the server before the context).  Each
 * turn it (1) admits waiting requests in arrival order while the sum of their
 * resident footprints (the matrix copied into HBM, 8 n^2 bytes plus 4 KiB)
 * stays within hbm_budget_bytes (0: 16 GiB; a request larger than the budget
 * is admitted alone); (2) runs one round of the early-terminated CRA loop
 * (Section 2.1, Alg. 2.1; rounds as in det_batch) for every admitted request
 * of order <= 512, all their LU items in one persistent launch, each request
 * taking its residues as they arrive and completing when it early-terminates
 * or reaches the Hadamard bound; (3) runs one admitted request of larger order
 * by the introspective scheme of det_introspective (Section 4).  Requests that
 * arrive meanwhile join the next turn.  Request i's primes come from the
 * stream seeded by opts->seed + i, so its result is the same alone and in any
 * mix.  Budget and occupancy are reported by det_server_stats.
 */
typedef struct det_server det_server;
typedef struct {
  int64_t submitted, completed, waiting, admitted, max_admitted;
  int64_t rounds;          /* engine turns */
  int64_t queue_items;     /* (matrix, prime) LU items run through the queue */
  int64_t hbm_budget, hbm_in_use, hbm_peak;   /* bytes of admitted resident data */
} det_server_report;

det_status det_server_create(det_ctx *ctx, size_t hbm_budget_bytes, const det_opts *opts,
                             det_server **out);
/* Copies A (host or device, row-major n x n, leading dimension lda, |a| < 2^31)
 * and queues it; *request_id identifies it.  Returns at once. */
det_status det_server_submit(det_server *s, const int64_t *A, int64_t n, int64_t lda,
                             int64_t *request_id);
/* *done = 1 when the request has finished (waits up to timeout_ms for it; -1:
 * without limit, 0: no wait); then sign, |det| as little-endian limbs in
 * mag[0 .. *limb_count) (DET_E_BUFFER_TOO_SMALL with *limb_count set when
 * limb_cap is too small) and the latency from submission to completion in ms.
 * A request that failed returns its status. */
det_status det_server_poll(det_server *s, int64_t request_id, int timeout_ms, int *done,
                           int *sign, uint32_t *mag, int64_t limb_cap, int64_t *limb_count,
                           double *latency_ms);
det_status det_server_stats(det_server *s, det_server_report *out);
/* Finishes every submitted request, stops the engine and frees the server. */
void det_server_destroy(det_server *s);

/*
 * Kernel timing (measurement support, not part of the method).  After
 * det_profile_select(ctx, kind), every launch of that kernel class made by
 * the context is bracketed by HIP events recorded on the context's stream;
 * det_profile_read synchronizes the stream and returns the number of timed
 * launches, their summed duration in ms, and the algorithmic bytes and
 * arithmetic operations of those launches as the launcher counted them from
 * its shapes (operations: 2 per modular multiply-add for the FP64 and
 * lifting kernels, 2 per int8 multiply-add for the int8 limb products).
 * The counters are then reset.  DET_KERNEL_NONE stops timing.
 */
typedef enum {
  DET_KERNEL_NONE = 0,
  DET_KERNEL_LIFT_X = 1,     /* x_i = A^{-1} r_i mod p                  */
  DET_KERNEL_LIFT_R = 2,     /* r_{i+1} = (r_i - A x_i) / p             */
  DET_KERNEL_GEMM_F64 = 3,   /* trailing update on FP64 MFMA            */
  DET_KERNEL_GEMM_I8 = 4,    /* trailing update on int8 MFMA (3 limbs; the limb splits included) */
  DET_KERNEL_PANEL = 5,      /* panel factorisation                     */
  DET_KERNEL_TRSM = 6,       /* in-place triangular apply               */
  DET_KERNEL_TRI_INV = 7,    /* diagonal-block triangular inverse       */
  DET_KERNEL_RESIDUES = 8,   /* A mod p for a batch of primes           */
  DET_KERNEL_LIFT = 9        /* all lifting steps in one cooperative launch */
} det_kernel;

det_status det_profile_select(det_ctx *ctx, det_kernel kind);
det_status det_profile_read(det_ctx *ctx, int64_t *launches, double *total_ms, double *bytes,
                            double *ops);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_CS_0511066_AMD_DET_H */
