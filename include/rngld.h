/*
 * rngld.h -- C ABI of librngld: random numbers generated on the fly inside a Langevin-dynamics
 * step, on AMD MI355X (gfx950).
 *
 * Method: Zhmurov, Rybnikov, Kholodov & Barsegov, "Efficient pseudo-random number generators for
 * biomolecular simulations on graphics processors" (arXiv:1003.1123).  Generators: Hybrid Taus
 * (Sec. II.D, Appendix A Alg. 1) and Ran2 (Sec. II.C, Alg. 2), one generator per thread
 * (Sec. III.B); additive lagged Fibonacci mod 2^32 (Sec. II.E Eq. 3, Alg. 3, Table I), one
 * generator shared by all threads (Sec. III.C).  Box-Muller turns uniforms into Gaussian forces
 * (Sec. I, II.A); four uniforms feed the three force components of one oscillator-step
 * (Table II caption).  The LD model is N independent 3-D harmonic oscillators in a stochastic
 * thermostat (Sec. IV).
 *
 * Conventions for every entry point:
 *  - returns RNGLD_OK (0) or a negative RNGLD_E* code; never throws; the message of the last
 *    failure on the calling thread is rngld_last_error();
 *  - all arguments are validated on the host before anything is enqueued; a failed call enqueues
 *    nothing (except RNGLD_EHIP, raised by the HIP runtime while enqueueing);
 *  - pointers prefixed d_ are device memory owned by the caller; h_ are host memory read during
 *    the call only; nothing is allocated or freed (ld_autotune is the one exception, see there);
 *  - work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and the call returns
 *    without synchronising; calls on one state buffer must be ordered by the caller;
 *  - all integer words are little-endian uint32; floating point is IEEE binary32 unless stated.
 */
#ifndef RNGLD_H
#define RNGLD_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define RNGLD_API __attribute__((visibility("default")))
#else
#define RNGLD_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------------------------- */
#define RNGLD_OK 0
#define RNGLD_EINVAL (-1)  /* null pointer, unknown kind, inconsistent sizes or parameters */
#define RNGLD_ELAG (-2)    /* lagged-Fibonacci lags / wave / ring unusable (see rngld_cfg) */
#define RNGLD_ESIZE (-3)   /* a caller buffer is smaller than required */
#define RNGLD_EHIP (-4)    /* the HIP runtime reported an error */
#define RNGLD_ENOTSUP (-5) /* valid request that this library does not implement */

/* ---- generator kinds ------------------------------------------------------------------------ */
#define RNGLD_HYBRID_TAUS 0 /* Sec. II.D, Alg. 1: three taus88 components xor an LCG (Eq. 1) */
#define RNGLD_RAN2 1        /* Sec. II.C, Alg. 2: two L'Ecuyer LCGs + 32-entry Bays-Durham table */
#define RNGLD_LAGFIB 2      /* Sec. II.E, Alg. 3: y_n = y_{n-ll} + y_{n-sl} mod 2^32, shared */
#define RNGLD_LCG 3         /* Sec. II.B, Eq. 1: Quick-and-Dirty LCG x = a x + c mod 2^32, per thread */
#define RNGLD_NO_NOISE 4    /* no generator: the LD step with a zero random force, i.e. the
                               deterministic dynamics alone (Fig. 6's "dynamics without RNG").
                               Bit-identical to a run with kT = 0 under any generator.  No state
                               (0 bytes, d_state may be NULL, n_streams is ignored); rng_init and
                               rng_init_ensembles do nothing; rng_uniform and rng_gaussian return
                               RNGLD_ENOTSUP; ld_step, ld_run and plans run; the adjoint does not. */

/*
 * Generator configuration.
 *  seed        : 64-bit seed.  Per-thread kinds: word i of global stream j is the high half of
 *                SplitMix64's mix(seed + (4j + i + 1) * 0x9E3779B97F4A7C15); LF: the window
 *                y_{-ll+i} = LCG^{i+1}(word 0 of stream 0), LCG of Eq. 1.
 *  n_streams   : per-thread kinds: number of streams (= oscillators) the state holds, S.
 *  stream_base : per-thread kinds: global index of the state's stream 0 (seeding only; lets
 *                a state hold any contiguous range of one seed's streams).
 *  lf_ll/lf_sl : LF long and short lag, 0 < sl < ll < 2^31 (Table I lists usable pairs).
 *  lf_wave     : LF wave width W, positions generated concurrently; 0 selects sl.  Rounded down
 *                to a multiple of 4.  Must satisfy 4 <= W <= sl (RNGLD_ELAG otherwise).  Results
 *                do not depend on W.
 *  lf_ring     : LF ring length R in words; 0 selects 2 (ll + sl), or ll + sl when 2 (ll + sl)
 *                reaches 2^30.  Must satisfy ll + W <= R < 2^31.  A fused LD run uses one
 *                persistent launch when sl >= 256 and its own copy of the sequence (about
 *                2 (ll + sl) words, each sl-long link padded to a 256-byte boundary, in the
 *                workspace) stays below 2^29 words; it reads the state's last ll values at the
 *                start and writes the new last ll values back at the end, so its result does not
 *                depend on R.
 *  lcg_leap    : LCG only.  0: stream j starts from its own seed word (word 0 of stream j).  L > 0:
 *                the streams divide one sequence (cycle division, Sec. III): stream j starts at
 *                position j * L of the sequence from word 0 of stream 0.  Eq. 1 has a single cycle
 *                of 2^32, so every stream is a shift of the same sequence; L = 4 makes stream j + 1
 *                the same as stream j one LD step later (the inter-stream correlation of Fig. 4b).
 *  lf_discard  : LF only, at most 2^40.  rng_init generates the first lf_discard values of the
 *                sequence from the seeded window and drops them (a warm-up of the initial seeds of
 *                Alg. 3): value n of the seeded state is then value lf_discard + n of the sequence
 *                without discard.  0 (default) keeps the window as seeded.
 */
typedef struct rngld_cfg {
    int32_t kind;
    uint32_t lf_ll;
    uint32_t lf_sl;
    uint32_t lf_wave;
    uint64_t seed;
    uint64_t n_streams;
    uint64_t stream_base;
    uint64_t lf_ring;
    uint64_t lcg_leap;
    uint64_t lf_discard;
} rngld_cfg;

/*
 * State buffer layouts (part of the ABI; a byte copy of the state is a checkpoint):
 *  HYBRID_TAUS : uint32 z[4][S], component-major: z[c*S + j] is word c of stream j
 *                (c = 0..2 Tausworthe components, 3 = LCG).                 16*S bytes.
 *  RAN2        : int32 r[35][S]: row 0 idum, 1 idum2, 2 iy, 3+t iv[t] (t = 0..31).  140*S bytes.
 *  LCG         : uint32 x[S].  4*S bytes.
 *  NO_NOISE    : none.  0 bytes.
 *  LAGFIB      : 64-byte header { uint64 pos; uint32 slot; uint32 ll, sl, R, W; ... } followed by
 *                uint32 ring[R]; y_n lives in ring[(slot + n - pos) mod R] for the last ll
 *                positions n < pos.  pos counts values generated since rng_init.  Then, from the
 *                next 128-byte boundary, working words of the persistent stream runs: a status
 *                word (nonzero after a run that gave up waiting; its output is then invalid) and
 *                2 x 8192 progress words 128 bytes apart, undefined between calls.  Then, when
 *                sl >= 256 and it is addressable (nr slp < 2^29 words, nr sl < 2^31), from the
 *                next 256-byte boundary the Gaussian stream run's own ring: nr = ceil(2 (ll + sl)
 *                / sl) links of slp = sl rounded up to 64 words, undefined between calls.
 *                align128(64 + 4 R) + 128 + 2 * 8192 * 128 bytes, + the ring's 4 nr slp bytes
 *                (256-byte aligned) when present.
 */
RNGLD_API int rngld_state_bytes(const rngld_cfg *cfg, size_t *bytes);

/* Seed the state (Sec. III.B seeding, Alg. 2 initialisation for Ran2, Alg. 3 window for LF, then
 * lf_discard values of the LF sequence generated and dropped). */
RNGLD_API int rng_init(const rngld_cfg *cfg, void *d_state, size_t state_bytes, void *stream);

/*
 * Bare generator output (no dynamics), advancing the state: the streams of Sec. III.B (one
 * generator per thread) and the shared sequence of Sec. III.C (Alg. 3), without the LD step.
 *  per-thread kinds: per_stream values of every stream, d_out[t*S + j] = value t of stream j;
 *                    out_len >= per_stream*S.  Taus: the xor word; Ran2: iy in [1, 2147483562].
 *  LAGFIB          : per_stream consecutive values of the one sequence, d_out[n] = y_{pos+n};
 *                    d_out doubles as the lag table for the values it holds.  With sl >= 4096
 *                    and at least 4 sl values (and no stream capture), one persistent launch
 *                    generates them; otherwise one launch per wave of W values.
 */
RNGLD_API int rng_uniform(const rngld_cfg *cfg, void *d_state, size_t state_bytes, uint64_t per_stream,
                uint32_t *d_out, uint64_t out_len, void *stream);

/*
 * Gaussian output by the Box-Muller transform (Sec. I; Sec. II.A on turning uniform variates into
 * other distributions): values 2i and 2i+1 of a stream are r cos(2 pi u1), r sin(2 pi u1) with
 * r = sqrt(-2 ln u0), u0 = ((w0 >> 8) + 1) 2^-24, u1 = (w1 >> 8) 2^-24 from that stream's words
 * 2i and 2i+1 (Ran2 word: (iy - 1) << 1).  per_stream must be even.  Layout as rng_uniform.
 * LAGFIB: with a 16-byte aligned d_out and at least 16 n values (n = 64 x the consumer waves of
 * the persistent run, x 1, 2 or 4), one persistent producer/consumer launch generates the first
 * 4 n T of them, T = per_stream / (4 n): producers extend the sequence in the state's own ring as
 * in the fused LD run and consumers write the Box-Muller pairs once; the rest continue as below.
 * Other calls that take rng_uniform's persistent launch are generated as integers into d_out (as
 * the lag table) and then transformed pair by pair in place.
 */
RNGLD_API int rng_gaussian(const rngld_cfg *cfg, void *d_state, size_t state_bytes, uint64_t per_stream,
                 float *d_out, uint64_t out_len, void *stream);

/*
 * The Box-Muller transform the generators apply (Sec. I), on caller-supplied word pairs:
 * d_out[2i] = r cos(2 pi u1), d_out[2i+1] = r sin(2 pi u1) with r = sqrt(-2 ln u0),
 * u0 = ((d_words[2i] >> 8) + 1) 2^-24, u1 = (d_words[2i+1] >> 8) 2^-24.  Lets the transform be
 * checked over its whole 24-bit input domain independently of any generator.
 */
RNGLD_API int rng_box_muller(const uint32_t *d_words, uint64_t n_pairs, float *d_out, void *stream);

/* ---- Langevin dynamics ------------------------------------------------------------------------ */
/*
 * Physical parameters (binary32).  scheme 0: underdamped (Sec. I), semi-implicit Euler-Maruyama
 *   v' = (1 - gamma dt) v - (k dt / m) x + sqrt(2 gamma kT dt / m) g,   x' = x + dt v'.
 * scheme 1: overdamped, Eq. (5) of Sec. IV with xi = m gamma:
 *   x' = x - (k dt / xi) x + sqrt(2 kT dt / xi) g   (v untouched).
 * Requires m > 0, gamma > 0, k >= 0, kT >= 0, dt > 0, all finite.
 * The step's coefficients (c = 1 - gamma dt, k dt / m, sqrt(2 gamma kT dt / m); for scheme 1
 * k dt / xi and sqrt(2 kT dt / xi)) are computed in double precision from these binary32 values
 * and rounded to binary32 once per call; so are the adjoint's partials dt / m, -dt and
 * s / (2 gamma), s / (2 kT) with s the double-precision noise amplitude.  A run iterates the map
 * with those rounded coefficients.
 */
typedef struct ld_params {
    float m, k, gamma, kT, dt;
    int32_t scheme;
} ld_params;

/* One ensemble of a (possibly batched) run: oscillators [offset, offset + n) of x, v and of the
 * generator state, with its own parameters; seed is used by rng_init_ensembles only. */
typedef struct ld_ensemble {
    uint64_t offset;
    uint64_t n;
    ld_params p;
    uint32_t pad;
    uint64_t seed;
} ld_ensemble;

/* Observables, recorded after t = 0, stride, 2*stride, ... <= n_steps steps of a run (stride 0 =
 * none), as means over the ensemble's 3n coordinates, 6 doubles per point:
 * <x^2>, <v^2>, <x v>, <x>, <x(t) x(t0)>, <v(t) v(t0)> (the last two are 0 for t < t0).  Sec. IV. */
typedef struct ld_obs {
    uint32_t stride;
    uint32_t t0;
} ld_obs;

#define RNGLD_NOBS 6

/*
 * Seed the per-thread state for batched runs: for each ensemble e, streams
 * [offset_e, offset_e + n_e) of the state are seeded as streams 0..n_e-1 of seed_e, so ensemble e
 * of a batched run reproduces a plain run of n_e oscillators with cfg.seed = seed_e.
 * cfg->seed and cfg->stream_base are ignored.  Per-thread kinds only.
 */
RNGLD_API int rng_init_ensembles(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                       uint32_t n_ens, void *stream);

/*
 * One LD step of n oscillators in the paper's protocol (Sec. IV; Fig. 5 caption): load x, v and
 * the generator state from device memory, draw four words per oscillator, update, store back.
 * d_x, d_v are float[3][n] component-major.  Per-thread kinds need n <= S.  LAGFIB: oscillator j
 * takes y_{pos + 4j + r}, r = 0..3 (Alg. 3), run as ceil(4n / W) dependent waves.
 */
RNGLD_API int ld_step(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_params *p, uint64_t n, float *d_x,
            float *d_v, void *stream);

/*
 * n_steps LD steps (the oscillators of Sec. IV, the step of ld_params) of n_ens ensembles (batched
 * when n_ens > 1) with the generator fused into the update, as Sec. III.A argues (numbers generated
 * inside the simulation kernel, not pre-generated), and x, v and the per-thread state held on chip
 * for the whole run.  ld_workspace_bytes sizes the caller's workspace for the same arguments.
 *  d_x, d_v   : float[3][n_total]; ensembles must lie inside [0, n_total) and must not overlap.
 *  obs, d_obs : optional observables, d_obs = double[n_ens][P][6], P = n_steps/stride + 1.
 *  d_ws       : workspace of ld_workspace_bytes() bytes (any alignment >= 256).  Its first four
 *               bytes are a uint32 status word: nonzero after a persistent lagged-Fibonacci run
 *               that gave up waiting for a dependency (the run's results are then invalid); the
 *               next four bytes say which lagged-Fibonacci path ran (1 = persistent, 2 = waves).
 *               Read them after synchronising the stream.
 * LAGFIB supports n_ens == 1 only (one shared sequence).  The result of ensemble e equals a plain
 * run (n_ens = 1, offset 0) on that ensemble alone, bit for bit, under the same tuning.
 */
RNGLD_API int ld_workspace_bytes(const rngld_cfg *cfg, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total,
                       uint32_t n_steps, const ld_obs *obs, size_t *bytes);
RNGLD_API int ld_run(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens, uint32_t n_ens,
           uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v, const ld_obs *obs, double *d_obs,
           void *d_ws, size_t ws_bytes, void *stream);

/*
 * Allocation-free ld_run, for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The same run as ld_run with the
 * same arguments, results and tuning, bit for bit, except that the workspace is not the caller's:
 * the library keeps one array of RNGLD_NOALLOC_SCRATCH_BYTES device bytes on every GPU it runs
 * on, from the first call on that GPU until the process ends, and the call allocates and frees
 * nothing.
 *  d_status : NULL, or caller-owned device memory for two uint32 words that receive what ld_run
 *             leaves in its workspace's first eight bytes (status word, lagged-Fibonacci path).
 * A run whose ld_workspace_bytes() exceeds RNGLD_NOALLOC_SCRATCH_BYTES is rejected with
 * RNGLD_ESIZE before anything is enqueued (e.g. long runs of many oscillators with observables;
 * a lagged-Fibonacci run with Table I's largest lags and no observables fits).
 * Every call on one GPU shares that GPU's array and leaves its contents behind; the run clears
 * what it needs cleared.  Calls that overlap in time on one GPU (other streams, other threads)
 * race on the array: order them on one stream, or use ld_run with separate workspaces.
 */
#define RNGLD_NOALLOC_SCRATCH_BYTES (48u * 1024u * 1024u)
RNGLD_API int ld_run_noalloc(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                   uint32_t n_ens, uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v, const ld_obs *obs,
                   double *d_obs, uint32_t *d_status, void *stream);

/* ---- tuning, hipGraph plans, autotuner ------------------------------------------------------ */
/*
 * Launch shape of the per-thread LD kernels.  block: threads per block (64, 128, 256 or 512);
 * osc_per_thread: 1 or 2; steps_per_launch: 0 = whole run in one launch; blocks_per_cu: 0 = one
 * block per tile, else a persistent grid of blocks_per_cu * CUs blocks striding over tiles.
 * block and osc_per_thread fix the reduction order of the observables.
 */
typedef struct ld_tuning {
    uint32_t block;
    uint32_t osc_per_thread;
    uint32_t steps_per_launch;
    uint32_t blocks_per_cu;
    uint32_t lf_waves; /* LAGFIB only: 0 = one persistent launch when the lags and ring allow it
                          (see lf_ring), 1 = one launch per wave */
} ld_tuning;

/* Tuning used by ld_run for a generator kind (process-wide; default {256, 1, 0, 0, 0}). */
RNGLD_API int ld_get_tuning(int32_t kind, ld_tuning *out);
RNGLD_API int ld_set_tuning(int32_t kind, const ld_tuning *t);

/*
 * Pick the fastest tuning for this workload (the batched runs of config 4: many ensembles of
 * uneven size) by measurement, and install it with ld_set_tuning:
 *  1. block size x oscillators per thread x blocks per CU (0, 4, 8), each timed on a proxy run of
 *     the same ensembles for min(n_steps, 128) steps in one launch;
 *  2. steps per launch (0 = one launch, 2500, 1000, 500) for the chosen shape, each timed as a
 *     hipGraph replay (as ld_plan_create records it) of a proxy run of min(n_steps, 2500) steps
 *     (halved while it would exceed 2e11 oscillator-steps); the fastest wins, a single launch
 *     unless splitting is at least 0.5% faster.
 * Timing uses a private stream.  This is set-up code, not the hot path: it allocates and frees its
 * own scratch device memory.  cache_path (may be NULL) names a text file of one line per workload,
 * keyed by device (architecture and compute units), kind, n_total, n_ens, n_steps and a hash of
 * every ensemble's size and scheme; a key found there is installed without measuring, a new
 * measurement replaces the key's line (the file is rewritten through a temporary file).
 */
RNGLD_API int ld_autotune(const rngld_cfg *cfg, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total,
                uint32_t n_steps, const char *cache_path, ld_tuning *out);

/* A captured hipGraph of one ld_run call (config-4 style batched runs); replaying it advances the
 * run by n_steps from the current x, v and state.  Arguments as ld_run; buffers must outlive it. */
typedef struct rngld_plan rngld_plan;
RNGLD_API int ld_plan_create(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                   uint32_t n_ens, uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v, const ld_obs *obs,
                   double *d_obs, void *d_ws, size_t ws_bytes, void *stream, rngld_plan **out);
RNGLD_API int ld_plan_launch(rngld_plan *plan, void *stream);
RNGLD_API int ld_plan_destroy(rngld_plan *plan);

/* ---- differentiation ------------------------------------------------------------------------ */
/*
 * Loss L_e = mean over steps t_begin..t_end (1 <= t_begin <= t_end <= n_steps) of <x^2>_e (mean
 * over the ensemble's 3n coordinates of the positions after t steps); checkpoints every K steps.
 * This differentiates the paper's LD model (Sec. I; the oscillators of Sec. IV) with the noise
 * held fixed; the paper itself computes no gradients.
 * flags: any of RNGLD_ADJ_REPLAY (ld_run_backward uses the replay path for every ensemble) and
 * RNGLD_ADJ_SPREAD (ld_run_backward also returns standard errors, see there).
 */
typedef struct ld_loss {
    uint32_t t_begin;
    uint32_t t_end;
    uint32_t K;
    uint32_t flags;
} ld_loss;

#define RNGLD_ADJ_REPLAY 1u
#define RNGLD_ADJ_SPREAD 2u

/* Checkpoint buffer: ceil(n_steps/K) + 1 records, record c = state at step min(c*K, n_steps)
 * (the last record is the state at the end of the run):
 * float x[3][n_total], float v[3][n_total], then the generator state in the layout above with
 * S = n_total, then float lam_x[3][n_total], lam_v[3][n_total]: the gradient of the
 * sum of x^2 over the loss window's steps after the record with respect to the record's x and v
 * (the loss adjoint the register-only backward of the segment starting there starts from),
 * written by ld_run_ckpt for ensembles that can take the register-only backward. */
RNGLD_API int ld_ckpt_bytes(const rngld_cfg *cfg, uint64_t n_total, uint32_t n_steps, uint32_t K, size_t *bytes);
RNGLD_API int ld_adjoint_workspace_bytes(const rngld_cfg *cfg, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total,
                               uint32_t n_steps, const ld_loss *loss, size_t *bytes);

/* Forward run that writes checkpoints and the losses d_loss[n_ens] (double).  Underdamped,
 * per-thread kinds.  x, v and the state advance as in ld_run.  For Hybrid Taus ensembles that can
 * take the register-only backward (with two or more segments and K <= 65536) the run is
 * segment-parallel: every Tausworthe step is linear over GF(2) and the LCG step affine, so each
 * K-step segment starts from its generator state jumped ahead by bit-matrix products, runs from a
 * zero state, and a join pass adds, in FP64, the response to the true start state (the LD step is
 * linear).  x and v then agree with a sequential run up to rounding, the noise bit for bit.
 * d_ws: ld_adjoint_workspace_bytes. */
RNGLD_API int ld_run_ckpt(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                uint32_t n_ens, uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v, const ld_loss *loss,
                void *d_ckpt, size_t ckpt_bytes, double *d_loss, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Reverse-mode pathwise gradient d_grad[n_ens][3] = (dL/dk, dL/dgamma, dL/dkT) (double) of the
 * losses of ld_run_ckpt; the noise of every step is regenerated bit-exactly.  d_ckpt is read only.
 * With RNGLD_ADJ_SPREAD in loss->flags d_grad is [n_ens][6]: the three gradients, then the
 * standard error of each, i.e. sd / sqrt(n) of the n per-oscillator contributions whose mean the
 * gradient is (the oscillators are independent, so this is the sampling error of the gradient
 * as an estimate of d E[L] / d theta).
 * Two paths, chosen per ensemble:
 *  - register-only (Hybrid Taus, Ran2): each K-step segment runs forward from the checkpoint at its
 *    start, with the generator, Box-Muller and update steps of the forward run, starting from the
 *    loss adjoint that ld_run_ckpt left in that checkpoint (the reverse recursion is linear with
 *    a constant step matrix, so the forward run can form it) and carrying the adjoint forward
 *    through the inverse of the reverse step (mu = lam_v / (1 - gamma dt), lam_x' = lam_x +
 *    (k dt/m) mu, lam_v' = mu - dt lam_x', less each step's own loss term).  Used when rounding
 *    errors cannot grow by more than 8 over K such steps (max over j <= K of the Frobenius norm
 *    of the inverse step matrix to the power j, for the ensemble's FP32 coefficients), e.g.
 *    gamma dt <= 0.02 at K = 100 and dt = 0.01.  The segments of an oscillator run concurrently
 *    and store nothing per step; a workspace record of 24 bytes per oscillator and segment
 *    collects each segment's share of the gradient.
 *  - replay: each segment is rerun forward from the checkpoint at its start into a scratch of
 *    9 floats per oscillator-step and swept backward from there (ensembles whose errors could
 *    grow more, or every ensemble with RNGLD_ADJ_REPLAY).
 * ld_adjoint_workspace_bytes is the workspace of both ld_run_ckpt and ld_run_backward (one buffer
 * serves both: the segment-parallel forward's 52 bytes per oscillator and segment and the
 * backward's scratch share their space).  It includes each path's scratch only when some ensemble
 * takes it, so it depends on the ensembles' parameters and the flags.
 */
RNGLD_API int ld_run_backward(const rngld_cfg *cfg, const void *d_ckpt, size_t ckpt_bytes, const ld_ensemble *h_ens,
                    uint32_t n_ens, uint64_t n_total, uint32_t n_steps, const ld_loss *loss, double *d_grad,
                    void *d_ws, size_t ws_bytes, void *stream);

/* ---- diagnostics ---------------------------------------------------------------------------- */
RNGLD_API const char *rngld_last_error(void);
RNGLD_API int rngld_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RNGLD_H */
