// internal.hpp -- structures shared by the kernel translation units and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rngld.h"
#include "device.hpp"
#include "lf_flow.hpp"

namespace rngld {

constexpr int kBulkBlock = 256;

// per-ensemble record in the workspace (64 bytes)
struct EnsDev {
    uint64_t offset;      // first oscillator / stream column
    uint64_t n;           // oscillators
    uint32_t tile_begin;  // first tile of this ensemble
    uint32_t n_tiles;
    LdCoef coef;
    uint32_t pad[2];
};
static_assert(sizeof(EnsDev) == 64, "EnsDev layout");

// arguments of the fused per-thread LD kernel
struct LdArgs {
    void *state;
    uint64_t S;           // state row stride (streams)
    float *x, *v;
    uint64_t NT;          // x, v row stride (n_total)
    const EnsDev *ens;
    uint32_t n_ens;
    uint32_t n_tiles;     // tiles over all ensembles
    uint32_t step_begin;  // run-relative steps [step_begin, step_end) of this launch
    uint32_t step_end;
    uint32_t n_steps;
    uint32_t stride;      // observation stride (0 = none)
    uint32_t t0;
    uint32_t P;           // observation points
    double *partials;     // [P][n_tiles][6]
    float *t0buf;         // [6][NT] x(t0), v(t0) carried between launches
};

// lagged-Fibonacci device header (first 64 bytes of the state)
struct LfHeader {
    uint64_t pos;   // values generated so far
    uint32_t slot;  // ring slot of position pos
    uint32_t ll, sl, R, W;
    uint32_t pad[9];
};
static_assert(sizeof(LfHeader) == 64, "LfHeader layout");

// ring of R 32-bit words: slot (hdr->slot + n - hdr->pos) mod R holds y_n
struct LfRing {
    const LfHeader *hdr;
    uint32_t *ring;
    uint32_t R, ll, sl;
};

// LF phase of an LD step: oscillators [osc_begin, osc_begin + osc_count) take the 4 * osc_count
// consecutive positions starting `off_mod` ring slots after the call's first position
struct LfLdPhase {
    LfRing L;
    uint32_t off_mod;
    uint32_t osc_count;
    uint64_t pos_rel;     // position of the wave's first number relative to the call's first
    uint64_t osc_begin;
    uint64_t N;           // x, v and t0buf row stride
    uint64_t n_osc;       // oscillators of the run
    float *x, *v;
    LdCoef coef;
    uint32_t step;        // run-relative step index of this phase
    uint32_t stride, t0;  // observation
    uint32_t tile_base;   // first partial slot of this phase
    uint32_t n_tiles;
    uint32_t pad;
    double *partials;     // [P][n_tiles][6]
    float *t0buf;         // [6][N]
};

// persistent dataflow LD run over the shared lagged-Fibonacci sequence (k_lf.hip)
// the persistent producer/consumer LD run (roles and waits: lf_flow.hpp)
struct LfFlowArgs {
    LfRing L;              // the state's ring (read by the copy kernels only)
    LfFlowGeom geom;       // waits, with R = nr sl
    uint32_t *pring;       // the run's own ring: nr links of slp words
    LfPadRing pr;
    float *x, *v;          // first oscillator of the run; row stride N
    float *t0buf;          // [6][N] x(t0), v(t0)
    double *partials;      // [P][pstride][6], one row entry per 64-oscillator tile
    uint32_t *prod;        // [producer wave * kLfFlagStride] links done, zero at launch
    uint32_t *cons;        // [consumer wave * kLfFlagStride] tiles done (Kc per step), zero at launch
    uint32_t *status;      // [0]: nonzero once a wait gave up (the run is then invalid)
    uint64_t N;
    uint64_t n;            // oscillators
    LdCoef coef;
    uint32_t n_steps;
    uint32_t stride, t0;   // observation
    uint32_t pstride;
    uint32_t spin_limit;   // polls of one wait before the run gives up
    uint32_t np;           // producer waves per block: the block's first np waves
    uint32_t *out;         // bare-stream modes: run position P to out[P] (16-byte aligned)
};
// what the consumers of a persistent run do with their words: drive the LD run, or write their
// Box-Muller pairs to out
constexpr int kFlowLd = 0, kFlowGauss = 1;

// persistent bare stream: out[0, count) = the next count values of the sequence, out doubling as
// the lag table
struct LfStreamArgs {
    LfRing L;              // the state's ring: the ll values before the call (read only)
    LfFlowGeom geom;       // sl, slice_log2 and Ptot = count are used
    uint32_t *out;         // doubles as the lag table
    uint32_t *prod;        // [slice * kLfFlagStride] links done, zero at launch
    uint32_t *status;      // nonzero once a wait gave up
    uint32_t lla, llb;     // ll = lla sl + llb
    uint32_t n_slices, n_links;
    uint32_t spin_limit;
    uint32_t pad;
};
// progress words the LAGFIB state reserves after its ring for the bare-stream runs (bytes): the
// status line, then one line per producer and one per consumer
constexpr size_t kLfStreamFlagBytes = 128 + 2 * static_cast<size_t>(8192) * 32 * sizeof(uint32_t);
hipError_t launch_lf_stream(const LfStreamArgs &a, uint32_t grid, uint32_t m, hipStream_t st);

// ---- adjoint (k_adj.hip) ---------------------------------------------------------------------------
struct AdjCoef {
    LdCoef f;         // forward coefficients
    float dkap_dk;    // h / m
    float dc_dgamma;  // -h
    float dsig_dgamma;
    float dsig_dkT;
    float inv_c;       // 1 / c = inv_c + inv_c_lo, for the register-only backward's mu = lam_v / c:
                       // the pair keeps the carried adjoint free of the systematic bias that a
                       // rounded reciprocal would compound over a segment's steps
    uint32_t reg_only;  // 1: register-only backward for this ensemble, 0: replay
    float inv_c_lo;
    // adjoint propagator over one whole K-step segment with no loss term: the adjoint (lam_x,
    // lam_v) of the state at a segment's start is phi * (adjoint at its end) + what the segment's
    // own loss terms contribute; phi = B^K with B = [[1 - kap h, -kap], [c h, c]], row-major
    float phi[4];
    // 1: the forward run writes the loss adjoint into each checkpoint record (the ensemble can take
    // the register-only backward; reg_only is this without RNGLD_ADJ_REPLAY)
    uint32_t lam;
    // 1: the forward run is segment-parallel (Hybrid Taus with lam): each K-step segment runs from
    // a zero state with the generator jumped to its start, and a join pass adds the response to
    // the true start state.  FP64, row-major, acting on (x, v) column vectors:
    uint32_t sp;
    double fk[4];     // F^K, F = [[1 - h kap, h c], [-kap, c]] the forward step matrix
    double flast[4];  // F^len of the last segment
    double bk[4];     // B^K = (F^K)^T (B = F^T), the adjoint step over a whole segment (phi in FP64)
    // sums over j = 1..K of a_j^2, a_j b_j, b_j^2 with (a_j, b_j) the first row of F^j, each term
    // formed from their FP32 values.  B^j e1 is the same row, so the segment's own adjoint uses the
    // same sums as its loss
    double full[3];
};

// width of the per-tile FP64 partials of the adjoint kernels: three sums and their squares
constexpr uint32_t kAdjPartW = 6;
// per (oscillator, segment) record of the segment-parallel register-only backward: FP64 rows
// [0, 3), the segment's three gradient sums
constexpr uint32_t kAdjSegD = 3;
// checkpoint rows of a record: x[3], v[3], the generator rows (4 for Hybrid Taus, 35 for Ran2), then
// the loss adjoint lam_x[3], lam_v[3] of the record's state (written by the forward run for
// ensembles with lam); AdjArgs::lam_row is the first adjoint row of the run's kind
constexpr uint32_t kCkptLamRow = 6 + 4;
constexpr uint32_t kCkptLamRowRan2 = 6 + 35;
// segment-parallel forward: per (oscillator, segment) FP32 rows of the zero-start run: x_end[3],
// v_end[3], sum of x^2 over the window steps, and per component sum a_j x_j and sum b_j x_j over
// them
constexpr uint32_t kFwdSegF = 13;
// per segment: the columns of the three Tausworthe components' jump matrices (3 x 32 words), the
// LCG's multiplier and increment, two words of padding
constexpr uint32_t kJumpWords = 100;

struct AdjArgs {
    void *state;  // forward: live state (stride S); unused by backward
    uint64_t S;
    float *x, *v;
    uint64_t NT;
    const EnsDev *ens;  // coef of EnsDev is unused here; adj holds per-ensemble coefficients
    const AdjCoef *adj;
    uint32_t n_ens, n_tiles;
    uint32_t n_steps, K;
    uint32_t t_begin, t_end;
    uint8_t *ckpt;
    uint64_t rec_bytes;  // bytes per checkpoint record
    uint32_t lam_row;    // first adjoint row of a record (kCkptLamRow or kCkptLamRowRan2)
    float *scratch;      // backward, replay path: [K][9][NT]
    double *seg_d;       // backward, register-only path: [nseg][kAdjSegD][NT]
    uint32_t *jump;      // forward, segment-parallel: [nseg][kJumpWords]
    float2 *coef;        //   [n_ens][K]: (a_j, b_j), the first row of F^j, j = 1..K
    float *fwd_seg;      //   [nseg][kFwdSegF][NT]
    double *partials;    // [n_tiles][kAdjPartW]: the loss (forward), or per-oscillator gradient
                         // sums and sums of squares (backward)
};

// forward with checkpoints: the segment-parallel kernels for ensembles with sp (any_sp), the
// sequential kernel for the others (any_seq)
hipError_t launch_ld_ckpt(int kind, const AdjArgs &a, bool any_sp, bool any_seq, hipStream_t st);
// backward: the replay kernel for ensembles with reg_only == 0, the register-only kernel (Hybrid
// Taus) for those with reg_only == 1
hipError_t launch_ld_adjoint(int kind, const AdjArgs &a, bool any_replay, bool any_reg_only, hipStream_t st);
// out[e][0, width) = sums of partial slots 0..width-1 over the ensemble's tiles / (3 n denom_steps);
// with spread, also out[e][width + q] = the standard error of the mean of slot q's per-oscillator
// values (slot width + q holding their squares)
hipError_t launch_adj_finalize(const double *partials, uint32_t n_tiles, uint32_t width, bool spread,
                               const EnsDev *ens, uint32_t n_ens, double denom_steps, double *out, hipStream_t st);

// ---- launchers (k_rng.hip) -------------------------------------------------------------------------
hipError_t launch_seed(int kind, void *state, uint64_t S, uint64_t seed, uint64_t stream_base, uint64_t col_offset,
                       uint64_t count, uint64_t leap, hipStream_t st);
hipError_t launch_bulk_uniform(int kind, void *state, uint64_t S, uint64_t per_stream, uint32_t *out,
                               hipStream_t st);
hipError_t launch_bulk_gaussian(int kind, void *state, uint64_t S, uint64_t per_stream, float *out, hipStream_t st);
hipError_t launch_box_muller(const uint32_t *words, uint64_t n_pairs, float *out, hipStream_t st);
hipError_t launch_box_muller_inplace(uint32_t *buf, uint64_t n_pairs, hipStream_t st);

// ---- launchers (k_ld.hip) --------------------------------------------------------------------------
hipError_t launch_ld_run(int kind, const LdArgs &a, const ld_tuning &t, uint32_t grid, hipStream_t st);
hipError_t launch_obs_finalize(const double *partials, uint32_t n_tiles, uint32_t P, const EnsDev *ens,
                               uint32_t n_ens, double *out, hipStream_t st);
hipError_t launch_ld_step(int kind, void *state, uint64_t S, const LdCoef &coef, uint64_t n, float *x, float *v,
                          hipStream_t st);
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st);
size_t ld_run_lds_bytes(int kind, const ld_tuning &t);
const void *ld_run_kernel_ptr(int kind, const ld_tuning &t);

// ---- launchers (k_lf.hip) --------------------------------------------------------------------------
hipError_t launch_lf_seed(void *state, uint32_t ll, uint32_t sl, uint32_t R, uint32_t W, uint64_t seed,
                          hipStream_t st);
hipError_t launch_lf_uniform_phase(const LfRing &L, uint32_t *out, uint64_t first, uint32_t count, hipStream_t st);
hipError_t launch_lf_ring_store(const LfRing &L, const uint32_t *out, uint64_t count, uint32_t base_mod,
                                hipStream_t st);
hipError_t launch_lf_gauss_phase(const LfRing &L, float *out, uint64_t first, uint32_t off_mod, uint32_t count,
                                 hipStream_t st);
hipError_t launch_lf_advance(LfHeader *hdr, uint64_t count, uint32_t count_mod, hipStream_t st);
// one wave (count <= W) of positions generated into the ring only, slots off_mod + t from the header's
hipError_t launch_lf_discard_phase(const LfRing &L, uint32_t off_mod, uint32_t count, hipStream_t st);
hipError_t launch_lf_ld_phase(const LfLdPhase &ph, hipStream_t st);
hipError_t launch_lf_observe(const LfLdPhase &ph0, uint32_t n_phases, uint64_t phase_osc, uint32_t point,
                             bool t0_now, hipStream_t st);

constexpr int kLfLdBlock = 256;
constexpr int kLfFlowBlock = 1024;          // 16 waves per block, one block per CU
constexpr int kLfFlowSliceMax = 1024;       // producer offsets per link (16 per lane)
constexpr uint32_t kLfFlowMaxWaves = 8192;  // progress words reserved per role
constexpr uint32_t kLfFlagStride = 32;       // words between progress words: one 128-byte line each
// launch the producer/consumer kernel for consumer waves of up to kc tiles each; `lds` bytes of
// dynamic LDS per block.  hipErrorCooperativeLaunchTooLarge if `grid` blocks cannot be co-resident.
hipError_t launch_lf_flow(const LfFlowArgs &a, uint32_t grid, uint32_t kc, uint32_t lds, hipStream_t st,
                          int mode = kFlowLd);
// copy the window y_{-ll..-1} before a persistent run from the state's ring into the run's ring,
// and afterwards the window y_{Ptot-ll..Ptot-1} back (slots relative to the run's first position;
// the header is advanced separately)
hipError_t launch_lf_pad_in(const LfRing &L, uint32_t *pring, const LfPadRing &pr, hipStream_t st);
hipError_t launch_lf_pad_out(const LfRing &L, const uint32_t *pring, const LfPadRing &pr, uint64_t Ptot,
                             hipStream_t st);
hipError_t launch_fill_u32(uint32_t *dst, uint64_t count, uint32_t value, hipStream_t st);

}  // namespace rngld
