// Device-side data layout shared by the step kernel and the host planner.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace modal {

constexpr int kWave = 64;        // CDNA wavefront width; one wave per workgroup
constexpr int kMaxModes = 1024;  // per instance
constexpr int kMaxGroups = kMaxModes / 4 / kWave;  // float4 groups per lane
constexpr int kSweepLoads = 4;  // float4 loads per lane per sweep of Ht rows
constexpr int kChipWaves = 8;   // waves of an on-chip (register-resident) workgroup
constexpr int kChipMaxRows = 12;  // in-plane rows per wave on the on-chip path
constexpr int kChipWaveModes = 4 * 64;  // modes of an instance stepped by one wave (no tensor)

enum : int { KIND_LINEAR = 0, KIND_TENSION = 1, KIND_VK = 2 };

// One instance (modal system).  Per-mode arrays are padded to ntp = round-up
// of nt to a multiple of 4 with zeros, so every lane works on float4 groups.
struct InstDev {
  int kind, nt, nin, ntp;
  long long h_off;     // float offset of Ht[nin][nt][ntp] in the tensor pool
  int mode_off;        // offset into the per-mode arrays (multiple of 4)
  int nslab;           // number of work units (workgroups) sharing it
  int ctr_off;         // first of its nslab arrival words (one per slab: the
                       // number of steps that slab has published)
  long long part_off;  // float offset of its partial forces [2][nslab][ntp]
  float kappa;         // TENSION
  int out_row;         // row of y
  long long e_off;     // offset into the excitation pool
  long long n_exc;     // excitation length (0 = none)
  // parity-blocked tensor (blk = 1): modes are stored grouped by class, class
  // i on rows [cls[i], cls[i+1]) (each a multiple of 4, ntp = cls[4]); in-plane
  // row n holds, for every class i, the block of rows of class i against
  // the columns of class j = jmap[n][i] & 7 (or nothing if jmap < 0), as wide
  // as class j, at float offset boff[n][i] from the instance's start; w is
  // the widest class.  A map entry also holds bit 3 (the block stands for its
  // transpose too), the rows per piece qs = min(rows, 256 / (width / 4)) in
  // bits 4..12 and the number of pieces from bit 13.
  int blk, w;
  int cls[5];
  int row_off;         // VK: offset of its in-plane rows in per-row pools
  long long jmap_off;  // int4 offset of the map [nin][2] (jmap[4], boff[4]) in its pool
};

// A slice of in-plane rows [row0, row1) of one instance, owned by one
// workgroup.  Each owner keeps a private copy of the instance state.
struct UnitDev {
  int inst, row0, row1, slab;
  int state_off;  // offset into the per-unit state arrays (multiple of 4)
  int qs;         // stored rows of Ht[n] per sweep of the wave
  int J;          // float4 loads per lane per sweep (kSweepLoads)
  int pad;
};

// Dynamic LDS of the step kernel: q^n [kMaxModes], per-wave partial forces
// [NW][kMaxModes] (NW > 1), a flag word (16 bytes), per-wave reduction
// buffers [NW][red_floats].
// LDS of one step workgroup: q^n of the current unit, a flag word, and one
// row-reduction region of red_floats per wave.  A wave that has finished its
// row sweep parks its partial force in the first ntp floats of its own region
// (red_floats >= 2 ntp for every instance), where wave 0 sums them.
// A workgroup that owns a single unit for the whole launch may also keep that
// unit's state and its instance's per-mode coefficients resident in LDS: 13
// arrays of res_stride floats after the reduction regions (X hi, X lo, d hi,
// d lo, m hi, m lo, p hi, p lo, r hi, r lo, b, c, lambda).
constexpr int kResArrays = 13;
// Exchange words of the waves that share an in-plane row (one-unit
// workgroups, whose waves divide the unit's row blocks rather than its rows):
// per wave two row slots, each with kXchVals partial scalars and the row
// index (an int stored in a float slot's bits), for at most 8 waves.
constexpr int kXchVals = 4;
constexpr int kXchWords = 8 * 2 * (kXchVals + 1);
struct StepLds {
  float *xs, *red, *res, *xch;
  int* flag;
};
__host__ __device__ inline size_t step_lds_bytes(int nw, int red_floats, int res_stride = 0) {
  return sizeof(float) * ((size_t)kMaxModes + 4 + kXchWords + (size_t)nw * red_floats +
                          (size_t)kResArrays * res_stride);
}
__host__ __device__ inline StepLds step_lds(float* base, int nw, int red_floats) {
  StepLds L;
  L.xs = base;
  L.flag = reinterpret_cast<int*>(base + kMaxModes);
  L.xch = reinterpret_cast<float*>(L.flag + 4);
  L.red = L.xch + kXchWords;
  L.res = L.red + (size_t)nw * red_floats;
  return L;
}

// LDS of one reverse-sweep workgroup: q^n and u^n of the current unit, a
// flag word, and one reduction region of red_floats per wave (three vectors
// per row, double-buffered); a finished wave parks J u, F and its tangent
// sum in the first 2 ntp + 1 floats of its region.
struct GradLds {
  float *xs, *us, *red, *xch;
  int* flag;
};
__host__ __device__ inline size_t grad_lds_bytes(int nw, int red_floats) {
  return sizeof(float) * (2 * (size_t)kMaxModes + 4 + kXchWords + (size_t)nw * red_floats);
}
__host__ __device__ inline GradLds grad_lds(float* base) {
  GradLds L;
  L.xs = base;
  L.us = base + kMaxModes;
  L.flag = reinterpret_cast<int*>(base + 2 * kMaxModes);
  L.xch = reinterpret_cast<float*>(L.flag + 4);
  L.red = L.xch + kXchWords;
  return L;
}

// Register layout of one instance on the on-chip path.  Lane p of every
// wave stands for mode perm[p] (-1: none); modes may be grouped by parity
// class (each class's lanes contiguous from a multiple of 4).  Wave w holds
// the in-plane rows row[w][r] (-1: none), all with the same column pattern:
// lane p multiplies, in each of them, the jl[w][p] consecutive lanes' modes
// from lane jb[w][p] (the one column class whose entries can be nonzero
// against p's class; for a tensor without classes, all nt modes from 0).
struct ChipMap {
  short perm[kWave];
  short row[kChipWaves][kChipMaxRows];
  unsigned char jb[kChipWaves][kWave];
  unsigned char jl[kChipWaves][kWave];
};

struct StepParams {
  const InstDev* inst;
  const int4* jmap;     // block maps of parity-blocked instances
  const UnitDev* unit;
  const int* wg_begin;  // [n_wg + 1] unit ranges per workgroup
  const float* H;       // tensor pool
  // per-mode float-float coefficients of d+ = m X - p d + r (f_ext - f)
  const float *m_hi, *m_lo, *p_hi, *p_lo, *r_hi, *r_lo;
  const float *c_out, *lam, *b_ext;
  const float* e_ext;
  // per-unit state (float-float X = q^n and d = q^n - q^{n-1})
  float *x_hi, *x_lo, *d_hi, *d_lo;
  float* part;              // partial forces of split instances
  unsigned int* ctr;        // arrival words of split instances' slabs (InstDev.ctr_off)
  int* flags;               // [0] barrier timeout, [1] non-finite state
  unsigned long long timeout_ticks;  // limit of a slab wait (100 MHz clock ticks)
  long long* step_base;     // absolute index of the next step (device)
  float* y;                 // output, y[row * y_stride + s]; NULL = none
  long long y_stride;
  int n_steps;              // steps of this launch
  int red_floats;           // LDS floats reserved for the reduction buffer
  int mode_floats;          // length of each per-mode array
  // > 0: every workgroup owns exactly one unit, and holds its state and
  // coefficients in LDS (kResArrays arrays of res_stride >= ntp floats) from
  // the start of the launch, writing the state back at its end
  int res_stride;
  // checkpoints of the float-float state at steps that are multiples of
  // ckpt_every: [slot][4][mode_floats] (X hi, X lo, d hi, d lo); NULL = none
  float* ckpt;
  int ckpt_every;
  // per-step record of q^n and d^n (fp32) for steps rec_base.. : [step][mode_floats]
  float *rec_x, *rec_d;
  long long rec_base;
  const ChipMap* chip;  // on-chip path: one map per instance
};

// Reverse (adjoint) sweep over a recorded segment of steps.
struct GradParams {
  const InstDev* inst;
  const UnitDev* unit;
  const int* wg_begin;
  const float* H;
  const float* Hd;  // tangent tensor pool (same layout as H) or NULL
  const float *m_hi, *m_lo, *p_hi, *p_lo, *r_hi, *r_lo;
  const float *c_out, *lam, *b_ext;
  const float* e_ext;
  const float *rec_x, *rec_d;  // recorded q^n, d^n of the segment
  long long seg_base;          // absolute step of rec row 0
  int seg_len;                 // steps in the segment (processed last to first)
  int mode_floats;
  const float* ybar;           // dL/dy [batch][ybar_stride], absolute steps
  long long ybar_stride;
  // adjoint state per unit: qb = dL/dq^{n+1}, db = dL/dd^{n+2} (float-float)
  float *qb_hi, *qb_lo, *db_hi, *db_lo;
  // per-unit accumulators, float-float pairs [10][state floats]:
  // m, p, r, c, s (u.F per mode), theta (per mode)
  float* acc;
  int state_floats;
  float* part;           // partial (J u, F) of split instances, [2][nslab][2 ntp] at 2 part_off
  unsigned int* ctr;
  int* flags;
  unsigned long long timeout_ticks;  // limit of a slab wait (100 MHz clock ticks)
  long long done_before;  // reverse steps completed before this launch
  int red_floats;
  // per-row record of -2 eta_n (V_n . u) for every reverse step of the
  // segment: [seg_len][rows_total] (rows of all VK instances); NULL = none
  float* rrec;
  int rows_total;
  // records for the full tensor gradient (NULL = none), in forward step order
  // like rec_x: u^n per mode [seg_len][mode_floats], and eta_n, V_n . u per
  // in-plane row [seg_len][2][rows_total]
  float* urec;
  float* trec;
};

// One instance's share of the full tensor gradient: out[n][i][j] (caller
// layout, n < nin, i, j < nt) -= sum over the segment's steps of
// ((V_n . u) q_i + eta_n u_i) q_j.
struct TGradJob {
  float* out;
  int nt, nin, mode_off, row_off;
};
constexpr int kTgTile = 64;   // output tile edge (i and j)
constexpr int kTgChunk = 16;  // steps staged in LDS per round

// ------------------------------------------------------------ shared tensor
// Batches whose instances share one coupling tensor up to a per-row scale
// (Ht_b[n] = s_b[n] H0[n]) run on the MFMA kernel: V0 = H0[n] X is a dense
// product with the instances as columns.  A workgroup of kSharedWaves waves
// owns 16 JT columns per wave (one group, one tensor) and runs every step
// without talking to other workgroups.
constexpr int kSharedWaves = 4;
constexpr int kSharedMaxKT = 4;  // modes per instance <= 16 kSharedMaxKT
constexpr int kSharedMaxNin = 64; // in-plane rows per instance on this path

struct SharedWg {
  long long a_off;  // packed tensor of the group (floats)
  int nin, nt;      // in-plane rows, modes
  int kt, kc;       // 16-row tiles and 4-wide K steps (the launch's; rows and
                    // columns past nt are zero)
};

struct SharedSlot {
  int out_row;      // output row, or -1 for an empty column
  int pad;
  long long e_off;  // excitation offset
  long long n_exc;
};

struct SharedParams {
  const SharedWg* wg;
  const SharedSlot* slot;    // [n_wg * cols]
  const float* A;            // packed tensors: [n][t][c][64] per group
  const float* s2;           // [n_wg][nin_max][cols] squared row scales
  int nin_max, cols, ktot;   // cols = 64 JT, ktot = 16 KT
  // per (column, mode), layout [n_wg * cols][ktot]
  float *x_hi, *x_lo, *d_hi, *d_lo;
  const float *m_hi, *m_lo, *p_hi, *p_lo, *r_hi, *r_lo, *c_out, *b_ext;
  const float* e_ext;
  float* y;
  long long y_stride;
  int n_steps;
  const long long* step_base;
  int* flags;
};
// LDS: two staged tensor rows (each padded to whole rounds of the
// workgroup's 16-byte loads), X of every wave in two layouts, squared row
// scales [nin][cols]
__host__ __device__ inline size_t shared_lds_bytes(int kt, int kc, int jt, int nin_max) {
  const size_t nt = 64 * kSharedWaves;
  const size_t row4 = (size_t)kt * ((kc + 3) / 4) * 64;
  const size_t na = (row4 + nt - 1) / nt;
  return 16 * 2 * na * nt +
         sizeof(float) * (2 * (size_t)kSharedWaves * 16 * kt * 16 * jt + (size_t)nin_max * 64 * jt);
}

// ---------------------------------------------------------- linear batches
constexpr int kLinWaves = 2;  // waves per closed-form workgroup
constexpr int kLinRun = 32;   // steps per lane (strided by 64)

// A float-float complex number: real and imaginary parts as (high, low)
// FP32 pairs whose sum carries about 48 bits.
struct FFc {
  float rh, rl, ih, il;
};

// One mode: both roots of z^2 - g z - p, their 64th powers, and the
// recurrence y(n + 64) = a y(n) - b y(n - 64) that every combination of the
// two root terms satisfies (a = Re(z1^64 + z2^64), b = Re((z1 z2)^64)), all
// float-float, rounded from the host's FP64 values.  conj: z2 = conj(z1),
// only root 1 is evaluated (its amplitude carries the factor 2).
struct LinMode {
  FFc z1, z2, s1, s2;
  float ah, al, bh, bl;
  int conj, pad[3];
};

// A run of output samples of one instance from one amplitude set: sample i
// (< len) is the sum over modes [m0, m1) of Re(P1 z1^(e0+i) + P2 z2^(e0+i)),
// written to out[out_off + i].
struct LinSeg {
  int m0, mc, m1, pad;  // modes [m0, mc) complex-conjugate pairs, [mc, m1) real pairs
  long long amp_off;
  long long e0;
  long long out_off;
  long long len;
};

// Per mode, what the amplitude sets are built from (float-float).
struct LinInit {
  FFc z1, z2, A, B, C;
  float ch, cl, bh, bl;  // output weight c and force weight b
  long long e_off, n_exc;
  int conj, pad[3];
};

struct LinForced {
  long long inst, e_off, n_exc;
};

}  // namespace modal
