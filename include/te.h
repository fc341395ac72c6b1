/*
 * te.h -- C ABI of the MI355X (gfx950) perturbative-triples library.
 *
 * The library evaluates the (T) correction of closed-shell CCSD(T) as given
 * in Fajen, Kelly, Hohenstein, Martinez, "Accelerating CCSD(T) on GPUs"
 * (arXiv 2512.01055), section "Implementation Details":
 *
 *   E(T) = sum_{i<=j<=k} (2 - d_ij - d_jk) sum_{abc} (W + V)^{abc}_{ijk} Z^{abc}_{ijk} / D^{abc}_{ijk}
 *
 * with W from Eq. 2 summed over the six pair permutations of Eq. 5, the
 * singles term V of Eq. 3, and D = e_i + e_j + e_k - e_a - e_b - e_c (Eq. 4
 * with the sign of the paper's energy-kernel figure). Integrals are
 * chemists' (pq|rs); the restricted sum over occupied triples is the same
 * number as Eq. 1's restricted sum over virtual triples.
 *
 * All functions are extern "C", never throw, and report through te_status.
 * A failing call leaves its output arguments untouched; te_last_error()
 * returns a message for the calling thread's most recent failure.
 * Different jobs may be used from different threads at once; calls on one
 * job must not overlap (they share its streams and slice cache).
 */
#ifndef TE_H
#define TE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum te_status {
  TE_OK = 0,
  TE_PENDING = 1,     /* te_poll: the job has not finished;
                         te_energy_checkpointed: triples remain           */
  TE_EINVAL = -1,     /* bad argument (sizes, NULL pointers, bad values)   */
  TE_ENOMEM = -2,     /* the job cannot fit in the HBM budget              */
  TE_EDEVICE = -3,    /* a HIP runtime call failed                         */
  TE_EBUSY = -4,      /* server shutting down / queue full / file in use   */
  TE_ENOTFOUND = -5,  /* unknown or already-collected ticket               */
  TE_ECANCELED = -6,  /* the server was destroyed before the job ran       */
  TE_EIO = -7         /* reading or writing a checkpoint file failed       */
} te_status;

/* Arithmetic of the W contractions (Eqs. 2 and 5). In every mode the
 * denominators, the singles term, each triple's partial sum and E(T) itself
 * are evaluated in FP64. */
typedef enum te_precision {
  TE_FP64 = 0,    /* FP64 MFMA                                                 */
  TE_FP32 = 1,    /* operands rounded to FP32, FP32 MFMA, FP32 accumulation    */
  TE_BF16X3 = 2,  /* operands split into 3 BF16 parts, 6 cross products,
                     FP32 accumulation                                         */
  TE_BF16X2 = 3,  /* 2 BF16 parts, 3 cross products, FP32 accumulation         */
  TE_FP16X2 = 4   /* operands scaled by a power of two per operand family and
                     split into 2 FP16 parts, 3 cross products, FP32
                     accumulation, unscaled at the end                          */
} te_precision;

typedef enum te_memkind { TE_MEM_HOST = 0, TE_MEM_DEVICE = 1 } te_memkind;

/* One closed-shell (T) problem, canonical orbitals. Every array is row-major
 * FP64 and every pointer lives in the memory named by `mem`.
 *
 *   eps_occ [o]            occupied orbital energies
 *   eps_vir [v]            virtual orbital energies
 *   t1      [o][v]         t1[i][a]       = t_i^a
 *   t2      [o][o][v][v]   t2[i][j][a][b] = t_ij^ab, equal to t2[j][i][b][a]
 *
 * Integrals, either as density-fitting / Cholesky factors (Eq. 6; naux > 0)
 *   B_oo [naux][o][o], B_ov [naux][o][v], B_vv [naux][v][v],
 *   (pq|rs) = sum_Q B^Q_pq B^Q_rs, B_oo and B_vv symmetric in their pair,
 * or, when naux == 0, explicitly
 *   ovvv [o][v][v][v] = (ia|bc),  ovoo [o][v][o][o] = (ia|jk),
 *   ovov [o][v][o][v] = (ia|jb).
 * Pointers of the unused form may be NULL.
 */
typedef struct te_problem {
  int32_t o, v, naux;
  te_memkind mem;
  const double *eps_occ, *eps_vir;
  const double *t1, *t2;
  const double *B_oo, *B_ov, *B_vv;
  const double *ovvv, *ovoo, *ovov;
} te_problem;

/* How (vv|vo) slices are held. */
typedef enum te_xmode {
  TE_X_AUTO = 0,        /* materialise all o*v^3 when it fits, else on the fly */
  TE_X_RESIDENT = 1,    /* materialise all slices at te_init                   */
  TE_X_ON_THE_FLY = 2   /* assemble slices from B_ov, B_vv into a slice cache;
                           the (ov|ov) blocks of Eq. 3 are then assembled per
                           triple instead of held as an o^2 v^2 array           */
} te_xmode;

typedef struct te_config {
  int device;           /* HIP device ordinal                                     */
  void *stream;         /* hipStream_t the work is ordered on; NULL: library-own  */
  size_t hbm_budget;    /* bytes the job may allocate; 0: 90% of free memory      */
  int validate;         /* 1: reject non-finite inputs and t2 asymmetry > 1e-12   */
  te_xmode x_mode;
  int x_cache_slices;   /* on-the-fly mode: slices kept resident; 0: automatic    */
  /* 1: t2 stays in host memory (for t2 larger than HBM). For each occupied
   * index a cache slot takes, its t2 panels (the column panel t2[:, p] and,
   * transposed, the row panel t2[p, :]) are copied in next to its (vv|vo)
   * slice. Needs the factors (naux > 0) and host arrays, and implies the
   * on-the-fly mode; t2 is borrowed until te_free. Results are bitwise those
   * of the resident layout. */
  int t2_host;
} te_config;

typedef struct te_stats {
  double seconds;        /* wall time of the call                                */
  double flops;          /* algorithmic W flops: n_triples * 12 v^3 (v + o)      */
  double tflops;         /* flops / seconds / 1e12                               */
  int64_t n_triples;     /* occupied triples evaluated                           */
  double stage_seconds;  /* part of `seconds` before the first launch: operand
                            conversion, scratch and slice-cache allocation,
                            planning (one-off set-up, not per triple)           */
  double assemble_flops; /* on-the-fly mode: flops spent assembling (vv|vo)
                            slices and per-triple (ov|ov) blocks               */
  /* Device time of the kernels, from HIP events recorded around each launch
   * on the stream it runs on: the W build (MFMA) and the energy consumer. */
  double w_kernel_seconds;
  int64_t w_launches;
  double e_kernel_seconds;
  int64_t e_launches;
  /* On-the-fly (vv|vo) mode: slices assembled, their device time (on a fill
   * stream of their own, beside the W builds: each slice is assembled once
   * the last W build that read its cache slot has finished, and before the
   * W builds that read it), and the number of slices the cache held. With
   * t2 in host memory the panel copies are part of the fills. The
   * per-triple (ov|ov) blocks run on the energy stream, overlapped with the
   * W build, and are not part of assemble_seconds. */
  int64_t slices_assembled;
  double assemble_seconds;
  int64_t cache_slices;
} te_stats;

typedef struct te_job_s *te_job;

/* Stage a problem on the device: the integrals of Eqs. 2 and 3 assembled
 * from the factors as Eq. 6 defines them, (pq|rs) = sum_Q B^Q_pq B^Q_rs --
 * (ia|jb) for the singles term, (ia|jk) for the occupied term of Eq. 2 and,
 * unless they are assembled on the fly, every (ia|bc) slice -- and padded
 * device layouts. Host arrays are copied before the call returns; device
 * arrays are read during the call and may be freed afterwards (in the
 * on-the-fly mode the job keeps its own copies of B_ov and B_vv), except t2,
 * which is borrowed (kept in use until te_free) when it is in device memory
 * and v is a multiple of 8, or when cfg->t2_host is set (host t2).
 * Errors: TE_EINVAL for o < 1, v < 1, v > 8184, naux < 0, NULL required
 * pointers, an inconsistent configuration or (validate) bad values;
 * TE_ENOMEM when the staged footprint exceeds the budget; TE_EDEVICE for HIP
 * failures. */
te_status te_init(const te_problem *prob, const te_config *cfg, te_job *out);

/* Evaluate E(T) of Eq. 1 over all occupied triples i<=j<=k (i=j=k
 * contribute zero and are skipped), in the form that carries Eq. 1's
 * restricted virtual sum over to the occupied labels: each triple's
 * sum_abc (W + V) Z / D weighted by 2 - d_ij - d_jk, with W from Eq. 2
 * summed over the permutations of Eq. 5, V from Eq. 3 and D from Eq. 4
 * (occupied minus virtual energies). Blocks until done. `per_triple` (host,
 * optional) receives the weighted partial of each triple in the order of
 * te_triple_list.
 * The result is bitwise reproducible for a given problem and precision.
 * The first call in a reduced precision converts the operands and keeps the
 * copy for later calls; a call in another reduced precision releases it
 * first, so a job holds at most one such copy. */
te_status te_energy(te_job job, te_precision prec, double *e_t, double *per_triple,
                    te_stats *st);

/* Evaluate only the listed triples: ijk is a host array [n][3] of
 * 0 <= i <= j <= k < o (not all equal). e_sum (optional) receives their
 * sum, per_triple (optional, host [n]) each weighted partial. */
te_status te_energy_triples(te_job job, te_precision prec, const int32_t *ijk, int64_t n,
                            double *e_sum, double *per_triple, te_stats *st);

/* te_energy_triples for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, results bitwise those of te_energy_triples
 * (same kernels, same launch items); st gets seconds, flops, tflops and
 * n_triples only. Allocates no device memory: the launch items, the W shares
 * of the batches in flight, the sextet partials and the per-triple results
 * live in one static device array of 512 MiB (one per device the call runs
 * on, held until the process ends). Needs a job staged by te_init with
 * resident (vv|vo) slices and t2 in device memory, and, for a reduced
 * precision, the operand copy an earlier te_energy / te_energy_triples call
 * in that precision made (TE_EINVAL otherwise). A list whose launch items
 * and per-triple results together with one triple's W shares (3 v^3 values
 * of 8 bytes in FP64, 4 otherwise, v rounded up to 8) exceed the array is
 * rejected with TE_EINVAL: in FP64 one triple's W fits for v up to 280, two
 * triples in flight (W build overlapping the energy) for v up to 216; FP32
 * and the split 16-bit modes (W in FP32) reach 352 and 280. The
 * array's contents persist between calls and are overwritten by each; calls
 * on one device are serialised inside the library (one process holds one
 * array per device, and two processes never share one). */
te_status te_energy_triples_noalloc(te_job job, te_precision prec, const int32_t *ijk,
                                    int64_t n, double *e_sum, double *per_triple,
                                    te_stats *st);

/* E(T) split by perturbation order into the two parts that make up the (T)
 * correction (its fourth- and fifth-order connected-triples terms, as the
 * introduction of the paper describes them): E[4] collects the W Z / D
 * terms of Eq. 1, which do not involve the singles, and E[5] the V Z / D
 * terms, V from Eq. 3 (linear in t1); E(T) = E[4] + E[5]. ijk / n as for
 * te_energy_triples; ijk == NULL takes every triple in te_triple_list order
 * (n is then ignored). e4_sum / e5_sum (optional) receive the two sums over
 * the triples, e4 / e5 (optional, host arrays of the triple count) each
 * triple's weighted parts. Errors as te_energy_triples. */
te_status te_energy_terms(te_job job, te_precision prec, const int32_t *ijk, int64_t n,
                          double *e4_sum, double *e5_sum, double *e4, double *e5,
                          te_stats *st);

/* Whole-job evaluation that survives interruption. The triples, in
 * te_triple_list order, are cut into chunks of `chunk` consecutive triples;
 * each finished chunk's per-triple E[4] and E[5] parts (te_energy_terms) are
 * appended to the checkpoint file at `path` as one checksummed record, and
 * the file is flushed to disk before the next chunk starts. A file left by
 * an earlier call with the same o, v, naux, precision, chunk and `tag` is
 * resumed: intact records are kept, a torn last record is dropped, and only
 * the missing chunks are evaluated. `tag` is any 64-bit value the caller
 * uses to name the inputs (a hash of them, say); a file whose header does
 * not match is rejected with TE_EINVAL and left as it is. max_chunks > 0
 * stops after that many newly evaluated chunks (runs under a wall-time
 * limit); 0 runs to the end. Returns TE_OK when every chunk is recorded,
 * with e_t / e4_sum / e5_sum (optional) set to the sums over all triples,
 * taken in triple order with compensation on the host: an interrupted and
 * resumed run gives the same bits as one that ran through. Returns
 * TE_PENDING while chunks remain (outputs untouched). st (optional)
 * describes the work of this call only. The call holds an exclusive
 * advisory lock (flock) on the file while it runs: a second call on the same
 * file, from this or another process, returns TE_EBUSY at once and leaves
 * the file as it is. File errors: TE_EIO. */
te_status te_energy_checkpointed(te_job job, te_precision prec, const char *path, uint64_t tag,
                                 int64_t chunk, int64_t max_chunks, double *e_t,
                                 double *e4_sum, double *e5_sum, te_stats *st);

/* Progress of a checkpoint file without a device or a job: checks its header
 * against the given problem (TE_EINVAL on a mismatch, TE_ENOTFOUND when the
 * file does not exist) and counts its intact chunk records. Reads only. */
te_status te_checkpoint_scan(const char *path, int32_t o, int32_t v, int32_t naux,
                             te_precision prec, uint64_t tag, int64_t chunk,
                             int64_t *chunks_done, int64_t *chunks_total);

te_status te_free(te_job job);

/* Number of triples i<=j<=k, not all equal: o(o+1)(o+2)/6 - o. */
int64_t te_num_triples(int32_t o);
/* Writes the triple list (i-major) into ijk [te_num_triples(o)][3]. */
te_status te_triple_list(int32_t o, int32_t *ijk);
/* Algorithmic flop count of one triple's W: 12 v^3 (v + o). */
double te_flops_per_triple(int32_t o, int32_t v);
/* On-the-fly mode planning: the number of (vv|vo) slice assemblies the
 * schedule performs for the full triple list of o occupied orbitals with a
 * cache of cache_slices (>= 3) slices and batches of up to `batch` triples.
 * Returns -1 for invalid arguments. */
int64_t te_plan_slice_loads(int32_t o, int32_t cache_slices, int32_t batch);

/* ---------------------------------------------------------------------
 * Serving: jobs of mixed (o, v) arrive while others run. The server admits
 * each job once its HBM footprint fits the budget, stages it, and packs its
 * triple work with that of the other resident jobs into shared launches.
 * A job's result is bitwise the same as te_energy would give alone.
 * te_submit / te_poll / te_wait may be called from any thread.
 * ------------------------------------------------------------------- */
typedef struct te_server_s *te_server;

typedef struct te_server_config {
  int device;
  size_t hbm_budget;      /* bytes for resident jobs; 0: 80% of free memory */
  int max_resident_jobs;  /* 0: 64                                           */
  int max_queued_jobs;    /* 0: 4096                                         */
  int borrow_inputs;      /* 0: te_submit copies the host arrays before it
                             returns; 1: it keeps the pointers, and the
                             caller keeps the arrays alive and unchanged
                             until the job's final te_poll / te_wait        */
  int staging_threads;    /* jobs staged concurrently; 0: 2                  */
} te_server_config;

te_status te_server_create(const te_server_config *cfg, te_server *out);
/* Queues a problem in host memory (copied, or borrowed with borrow_inputs)
 * for the E(T) of te_energy (Eq. 1 over i<=j<=k, Eqs. 2-6) in precision
 * `prec`; *ticket names it for te_poll / te_wait. Returns TE_ENOMEM if the
 * job could never fit the budget, TE_EBUSY if the queue is full or the
 * server is shutting down, TE_EDEVICE after a device failure. */
te_status te_submit(te_server srv, const te_problem *prob, te_precision prec,
                    uint64_t *ticket);
/* TE_PENDING while queued or running; the job's final status otherwise
 * (TE_OK with e_t = E(T) of Eq. 1, bitwise what te_energy gives for the same
 * problem and precision, and st filled in; st->seconds is the latency from
 * te_submit to completion). The ticket is released by the first final
 * answer; later polls return TE_ENOTFOUND. */
te_status te_poll(te_server srv, uint64_t ticket, double *e_t, te_stats *st);
/* te_poll that blocks until the job is final. */
te_status te_wait(te_server srv, uint64_t ticket, double *e_t, te_stats *st);
/* Stops the server; jobs not yet finished end with TE_ECANCELED. */
te_status te_server_destroy(te_server srv);

/* Diagnostic: the sustained matrix-core rate of `device` for the MFMA form
 * the W build uses in `prec` (FP64, FP32, BF16 or FP16 16x16 blocks), measured
 * with a register-only kernel that keeps every SIMD issuing independent
 * MFMA chains for about `seconds`. Puts a kernel's fraction of the published
 * peak in context (clocks under sustained matrix load sit below the peak
 * clock). Writes TFLOP/s of the instruction itself (for the split modes: per
 * product; BF16X3 and BF16X2 time the BF16 instruction, FP16X2 the FP16 one). */
te_status te_mfma_sustained(int device, te_precision prec, double seconds, double *tflops);

const char *te_strerror(te_status s);
const char *te_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TE_H */
