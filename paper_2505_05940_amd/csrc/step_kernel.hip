// Persistent time-stepping kernel for batches of modal systems (gfx950).
//
// A workgroup (one, four or eight 64-lane waves) owns a fixed list of work units
// for the whole launch; a unit is either a whole instance or a slab of
// in-plane rows of a von Karman instance whose coupling tensor is split over
// several workgroups; the waves of a workgroup share a unit's rows.  Per audio sample (paper: Sec. 3.2, modal oscillator
// update) each unit
//   1. publishes q^n (fp32 high part) to LDS and writes the output sample
//      y^n = sum_k c_k q_k^n (modal-to-physical transform at one point),
//   2. evaluates its share of the nonlinear modal force (Sec. 3.1):
//        von Karman, one pass over its rows of Ht:  V[n,k] = sum_j Ht[n][j][k] q_j
//        (Ht symmetric in its last two indices), eta_n = sum_k V[n,k] q_k,
//        F_k += eta_n V[n,k];
//        tension-modulated: F_k = kappa lambda_k q_k sum_j lambda_j q_j^2,
//   3. advances the state in float-float arithmetic in increment form
//        d^{n+1} = m q^n - p d^n + r (f_ext^n - F^n),  q^{n+1} = q^n + d^{n+1}
//      (m = g + p - 1 = -r omega^2 for Stormer-Verlet), where instances split
//      over several workgroups first exchange their partial forces through
//      global memory and wait until every slab of the instance has stored
//      its arrival word for the step.
// The coupling tensor is streamed from HBM once per step with 16-byte loads
// into registers, with the non-temporal hint for a batch (each element is
// used once per step) and the default policy for a latency plan, whose
// tensors stay in the caches from step to step.  LDS holds q^n and the
// cross-lane reduction of V.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "device_common.h"

namespace modal {

// -------------------------------------------------------- von Karman rows
// Rows [row0, row1) of one instance's Ht.  Row n is an nt x ntp matrix
// (nc = ntp/4 float4 per stored row), read as consecutive blocks of qs
// stored rows.  A block is contiguous, so lane slot v = lane + 64 j
// (j < kSweepLoads) reads float4 number v of the block: stored row
// q0 + v / nc, columns 4 (v % nc) .. +3; one sweep is a fully coalesced
// 4 KB read per wave.  Each block gets a buffer resource sized to the block,
// so idle slots (v >= qs nc) and the missing rows of the last block read
// zeros without touching memory.  Blocks are software-pipelined across rows:
// the loads of the next block are issued before the current one is used.
// At the end of a row the slot accumulators are reduced over the qs
// sub-rows through LDS (double buffered by row parity) into V[n, :] on the
// lanes owning each float4 column group (k4 = lane + 64 g), and eta_n and
// the force follow: F += eta_n V[n, :].  DEPTH buffers (2 or 3) keep
// DEPTH - 1 blocks' loads in flight; three serve small latency-bound units
// whose rows are only a block or two long.
template <int GM, int DEPTH, int POL>
__device__ void vk_rows(const float* __restrict__ Hb, int nt, int ntp, int qs, int row0,
                        int row1, const float* Xs, float* red, float4 (&Fa)[GM], int G,
                        int lane) {
  constexpr int J = kSweepLoads;
  if (row1 <= row0) return;
  const int nc = ntp >> 2;
  const int qsnc = qs * nc;
  int voff[J], sub[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int v = lane + kWave * j;
    voff[j] = 16 * v;
    sub[j] = v < qsnc ? v / nc : 0;
  }
  const int nblk = (nt + qs - 1) / qs;
  const long long blk_floats = (long long)qs * ntp;
  const long long row_floats = (long long)nt * ntp;
  const int blk_bytes = 4 * qs * ntp;
  const int last_bytes = 4 * (nt - (nblk - 1) * qs) * ntp;
  // position of the block being loaded ahead; past the last row the
  // resource covers zero bytes, so the (unconditional) loads return zeros
  // without a memory access and the loop keeps a single straight-line path
  int ln = row0, lb = 0;
  auto load = [&](float4 (&h)[J]) {
    const bool live = ln < row1;
    const float* bp = Hb + (live ? (long long)ln * row_floats + (long long)lb * blk_floats : 0);
    const int bytes = live ? (lb == nblk - 1 ? last_bytes : blk_bytes) : 0;
    const v4i r = buf_rsrc(bp, bytes);
#pragma unroll
    for (int j = 0; j < J; ++j) h[j] = buf_ld4<POL>(r, voff[j]);
    if (++lb == nblk) {
      lb = 0;
      ++ln;
    }
  };
  float4 ha[J], hb[J], acc[J];
#pragma unroll
  for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
  int n = row0, b = 0;
  // Uses block `hc` (row n, block b) after issuing the loads of the next
  // block into `hn`; returns false after the last row.  Two buffers used in
  // turn keep the next block's loads in flight while the current one is
  // consumed.
  auto step = [&](float4 (&hc)[J], float4 (&hn)[J]) -> bool {
    load(hn);
    const int q0 = b * qs;
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = fma4(hc[j], Xs[min(q0 + sub[j], nt - 1)], acc[j]);
    if (++b < nblk) return true;
    // row n complete: reduce over sub-rows, then eta_n and the force
    float* rb = red + (n & 1) * qs * ntp;
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (voff[j] < blk_bytes) st4(rb + (voff[j] >> 2), acc[j]);
    wave_lds_sync();
    float eta = 0.f;
    float4 V[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      V[g] = f4(0.f);
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) {
        const float4 s = sum_strided4(rb + 4 * k4, qs, ntp);
        V[g] = s;
        eta += dot4(s, ld4(Xs + 4 * k4));
      }
    }
    eta = wave_sum(eta);
#pragma unroll
    for (int g = 0; g < GM; ++g) Fa[g] = fma4(V[g], eta, Fa[g]);
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
    b = 0;
    return ++n < row1;
  };
  load(ha);
  if (DEPTH == 2) {
    while (step(ha, hb) && step(hb, ha)) {
    }
  } else {
    float4 hx[J];
    load(hb);
    while (step(ha, hx) && step(hb, ha) && step(hx, hb)) {
    }
  }
}

// The dense sweep over a range of row blocks instead of whole rows: blocks
// [t0, t1) of the unit whose rows start at row0, block t being block t % nblk
// of row row0 + t / nblk.  Used when a workgroup owns a single unit and its
// waves share the unit's blocks evenly, so that a unit of fewer rows than
// waves keeps every wave busy.  A row that lies wholly in the range is
// finished here (eta_n V_n added to the force).  A row that the range cuts
// (at most its first and its last) gives only partial V and eta_n, which
// are linear in the blocks summed: the partial V is parked in `defer` (two
// slots of ntp floats) and the partial eta_n and the row index in the
// wave's exchange words (slot 0: a row the range enters mid-row, slot 1: a
// row it leaves mid-row; row -1 = unused), for vk_rows_finish.
template <int GM, int DEPTH, int POL>
__device__ void vk_rows_range(const float* __restrict__ Hb, int nt, int ntp, int qs, int row0, int t0,
                              int t1, const float* Xs, float* red, float4 (&Fa)[GM], int G, int lane,
                              float* defer, float* xv, int* xr) {
  constexpr int J = kSweepLoads;
  if (lane == 0) {
    xr[0] = -1;
    xr[1] = -1;
  }
  if (t1 <= t0) return;
  const int nc = ntp >> 2;
  const int qsnc = qs * nc;
  int voff[J], sub[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int v = lane + kWave * j;
    voff[j] = 16 * v;
    sub[j] = v < qsnc ? v / nc : 0;
  }
  const int nblk = (nt + qs - 1) / qs;
  const long long blk_floats = (long long)qs * ntp;
  const long long row_floats = (long long)nt * ntp;
  const int blk_bytes = 4 * qs * ntp;
  const int last_bytes = 4 * (nt - (nblk - 1) * qs) * ntp;
  // loader: block lt (flattened), row ln, block lb of that row
  int lt = t0, ln = row0 + t0 / nblk, lb = t0 % nblk;
  auto load = [&](float4 (&h)[J]) {
    const bool live = lt < t1;
    const float* bp = Hb + (live ? (long long)ln * row_floats + (long long)lb * blk_floats : 0);
    const int bytes = live ? (lb == nblk - 1 ? last_bytes : blk_bytes) : 0;
    const v4i r = buf_rsrc(bp, bytes);
#pragma unroll
    for (int j = 0; j < J; ++j) h[j] = buf_ld4<POL>(r, voff[j]);
    ++lt;
    if (++lb == nblk) {
      lb = 0;
      ++ln;
    }
  };
  float4 ha[J], hb[J], acc[J];
#pragma unroll
  for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
  int t = t0, n = row0 + t0 / nblk, b = t0 % nblk, bfirst = b;
  auto step = [&](float4 (&hc)[J], float4 (&hn)[J]) -> bool {
    load(hn);
    const int q0 = b * qs;
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = fma4(hc[j], Xs[min(q0 + sub[j], nt - 1)], acc[j]);
    ++t;
    if (++b < nblk && t < t1) return true;
    // the row, or the range's share of it, is summed
    float* rb = red + (n & 1) * qs * ntp;
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (voff[j] < blk_bytes) st4(rb + (voff[j] >> 2), acc[j]);
    wave_lds_sync();
    float eta = 0.f;
    float4 V[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      V[g] = f4(0.f);
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) {
        const float4 sv = sum_strided4(rb + 4 * k4, qs, ntp);
        V[g] = sv;
        eta += dot4(sv, ld4(Xs + 4 * k4));
      }
    }
    eta = wave_sum(eta);
    if (bfirst == 0 && b == nblk) {
#pragma unroll
      for (int g = 0; g < GM; ++g) Fa[g] = fma4(V[g], eta, Fa[g]);
    } else {
      const int slot = bfirst > 0 ? 0 : 1;
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        const int k4 = lane + kWave * g;
        if (g < G && k4 < nc) st4(defer + slot * ntp + 4 * k4, V[g]);
      }
      if (lane == 0) {
        xv[slot] = eta;
        xr[slot] = n;
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
    b = 0;
    bfirst = 0;
    ++n;
    return t < t1;
  };
  load(ha);
  if (DEPTH == 2) {
    while (step(ha, hb) && step(hb, ha)) {
    }
  } else {
    float4 hx[J];
    load(hb);
    while (step(ha, hx) && step(hb, ha) && step(hx, hb)) {
    }
  }
}

// Completes the rows that vk_rows_range left to several waves, after a
// workgroup barrier: eta_n is the sum of the partials of every wave that
// holds row n (in wave order), and each of those waves adds eta_n times its
// partial V_n.  xv, xr: the exchange words of all nw waves (this wave's at
// 2 wave).
template <int GM>
__device__ void vk_rows_finish(const float* xv, const int* xr, int nw, int wave, int ntp,
                               const float* defer, float4 (&Fa)[GM], int G, int lane) {
  const int nc = ntp >> 2;
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int n = xr[2 * wave + slot];
    if (n < 0) continue;
    float eta = 0.f;
    for (int i = 0; i < 2 * nw; ++i)
      if (xr[i] == n) eta += xv[i];
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) Fa[g] = fma4(ld4(defer + slot * ntp + 4 * k4), eta, Fa[g]);
    }
  }
}

// ---------------------------------------------- parity-blocked von Karman rows
// Rows [row0, row1) of an instance stored parity-blocked: modes are grouped
// by class (class i on internal modes [cls[i], cls[i+1])), and in-plane row
// n holds, per class i, the rows of class i against the columns of class
// j = jmap[n][i] only (every other entry of those rows is zero), as a block
// as wide as class j (padded to 4) at its own offset (the second int4 of the
// row's map entry).  The sweep is the dense one applied to each (n, i) block
// in turn: pieces of qs = min(rows, 256 / (width / 4)) stored rows, lane slot
// v = lane + 64 j reading float4 v of the piece (sub-row v / (width / 4)),
// buffer resources sized to the valid rows, the next piece's loads issued
// before the current one is used.  Accumulating along the
// stored rows of block (n, i) gives V[n, k] for the modes k of class j
// (Ht symmetric), so at the end of each block the slot accumulators are
// reduced over the qs sub-rows through LDS onto the lanes owning those
// modes; at the end of row n, eta_n and the force follow as in the dense
// sweep.  The loader walks (n, i, block) one block ahead of the arithmetic
// and hands each block's target range and end-of-class/row flags along;
// each block's loads are issued before the previous one is used.
// When an in-plane row's blocks come in transposed pairs ((i, j) and (j, i),
// i != j) only (i, j) is stored (jmap entry j | 8): its stored rows also
// give V for class i by row dot products with q over class j, reduced over
// each row's float4 groups through LDS and collected per row in an LDS
// vector (vrow) that joins V at the end of the in-plane row.
struct BlkMeta {
  int q0;     // first stored row (internal mode) of the block
  int tc;     // first float4 column group of the target class
  int tlen;   // float4 column groups of the target class
  int flags;  // 1: last block of its class, 2: last of its row, 4: last overall,
              // 8: the block also stands for its transpose (row dot products)
  int rows;   // valid stored rows in the block
  int qs;     // sub-rows of the block's slot layout (256 / tlen, at most the class)
};

__device__ __forceinline__ int sel4(const int4 v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

template <int GM>
__device__ void vk_rows_blk(const float* __restrict__ Hb, const int4* __restrict__ jm,
                            const InstDev& I, int row0, int row1, const float* Xs,
                            float* red, float4 (&Fa)[GM], int G, int lane) {
  constexpr int J = kSweepLoads;
  constexpr int kSlotFloats = 4 * J * kWave;  // floats of one piece's slot layout
  if (row1 <= row0) return;
  const int ntp = I.ntp;
  const int nc_modes = ntp >> 2;
  // class boundaries (a private array; read through selects instead, it left
  // scratch but measured 9 % slower on the 256-plate batch)
  int cb[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) cb[i] = I.cls[i];
  auto co = [&](int i) { return cb[i]; };
  // one piece's slot layout for the class-end reductions (a wave's LDS
  // operations complete in order, so one buffer serves them all)
  float* rd = red + kSlotFloats;  // [kSweepLoads * 64] per-slot row dot partials
  float* vrow = rd + J * kWave;       // [ntp] row-dot part of V for the current row
  for (int k = lane; k < ntp; k += kWave) vrow[k] = 0.f;
  // loader position: row ln, class li, piece lb; jv, jo = map entries and
  // block offsets of row ln
  int ln = row0, li = 0, lb = 0;
  int4 jv = jm[2 * row0], jo = jm[2 * row0 + 1];
  auto has_block = [&](int i) { return co(i + 1) > co(i) && sel4(jv, i) >= 0; };
  // a paired block's partner (-1) is skipped like an empty one
  auto next_row = [&]() {
    if (++ln < row1) {
      jv = jm[2 * ln];
      jo = jm[2 * ln + 1];
    }
  };
  auto to_data = [&]() {  // first (row, class) at or after (ln, li) with a block
    while (ln < row1) {
      while (li < 4 && !has_block(li)) ++li;
      if (li < 4) return;
      next_row();
      li = 0;
    }
  };
  to_data();
  if (ln >= row1) return;  // no stored block in these rows
  auto load = [&](float4 (&h)[J], BlkMeta& m) {
    const bool live = ln < row1;
    const float* bp = Hb;
    int bytes = 0;
    m = BlkMeta{0, 0, 0, 0, 0, 1};
    if (live) {
      const int R = co(li + 1) - co(li);
      const int je = sel4(jv, li);
      const int tj = je & 7;
      m.tc = co(tj) >> 2;
      m.tlen = (co(tj + 1) - co(tj)) >> 2;
      m.qs = (je >> 4) & 511;  // min(R, 256 / tlen), from the map entry
      const int nb = je >> 13;  // pieces of the block
      m.q0 = co(li) + lb * m.qs;
      m.rows = min(m.qs, R - lb * m.qs);
      bp = Hb + sel4(jo, li) + (long long)lb * m.qs * 4 * m.tlen;
      bytes = 16 * m.rows * m.tlen;
      if (je & 8) m.flags = 8;
      if (++lb == nb) {
        m.flags |= 1;
        lb = 0;
        ++li;
        while (li < 4 && !has_block(li)) ++li;
        if (li == 4) {
          m.flags |= 2;
          li = 0;
          next_row();
          to_data();
          if (ln >= row1) m.flags |= 4;
        }
      }
    }
    const v4i r = buf_rsrc(bp, bytes);
#pragma unroll
    for (int j = 0; j < J; ++j) h[j] = buf_ld4(r, 16 * (lane + kWave * j));
  };
  float4 ha[J], hb[J], acc[J], V[GM];
  BlkMeta ma, mb;
#pragma unroll
  for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
#pragma unroll
  for (int g = 0; g < GM; ++g) V[g] = f4(0.f);
  // consumes block `hc` after issuing the loads of the next block into `hn`
  auto step = [&](float4 (&hc)[J], const BlkMeta& mc, float4 (&hn)[J], BlkMeta& mn) -> bool {
    load(hn, mn);
    // sub-row of each slot in this block's layout: v / tlen (v < 256, so the
    // rounded reciprocal with half a slot of margin floors exactly)
    const float inv = __builtin_amdgcn_rcpf((float)mc.tlen);
    int sub[J];
#pragma unroll
    for (int j = 0; j < J; ++j) sub[j] = (int)(((float)(lane + kWave * j) + 0.5f) * inv);
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = fma4(hc[j], Xs[min(mc.q0 + sub[j], ntp - 1)], acc[j]);
    if (mc.flags & 8) {
      // transposed contribution: V[q0 + t] += sum_c S[t][c] q[class j][c]
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int v = lane + kWave * j;
        const int c4 = min(v - sub[j] * mc.tlen, mc.tlen - 1);  // float4 column group of slot v
        rd[v] = dot4(hc[j], ld4(Xs + 4 * (mc.tc + c4)));
      }
      wave_lds_sync();
      if (lane < mc.rows) vrow[mc.q0 + lane] += sum_run(rd + lane * mc.tlen, mc.tlen);
    }
    if (mc.flags & 1) {
      // block row of class i done: reduce over sub-rows onto the target modes
      float* rb = red;
      const int wj = 4 * mc.tlen;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int v = lane + kWave * j;
        if (v < mc.qs * mc.tlen) st4(rb + 4 * v, acc[j]);
      }
      wave_lds_sync();
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        const int k4 = lane + kWave * g;
        const int c4 = k4 - mc.tc;
        if (g < G && c4 >= 0 && c4 < mc.tlen) {
          V[g] = add4(V[g], sum_strided4(rb + 4 * c4, mc.qs, wj));
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j) acc[j] = f4(0.f);
    }
    if (mc.flags & 2) {
      // row n done: V gets the row-dot part, then eta_n and the force
      wave_lds_sync();
      float eta = 0.f;
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        const int k4 = lane + kWave * g;
        if (g < G && k4 < nc_modes) {
          V[g] = add4(V[g], ld4(vrow + 4 * k4));
          st4(vrow + 4 * k4, f4(0.f));
          eta += dot4(V[g], ld4(Xs + 4 * k4));
        }
      }
      eta = wave_sum(eta);
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        Fa[g] = fma4(V[g], eta, Fa[g]);
        V[g] = f4(0.f);
      }
    }
    return !(mc.flags & 4);
  };
  load(ha, ma);
  while (step(ha, ma, hb, mb) && step(hb, mb, ha, ma)) {
  }
}

// Where one unit's state and its instance's per-mode coefficients live: in
// global memory, or resident in LDS for the whole launch.
struct ModeRefs {
  float *xh, *xl, *dh, *dl;
  const float *mh, *ml, *ph, *pl, *rh, *rl, *b, *c, *lam;
};

// Per-mode state update of the float4 groups owned by this lane; e is this
// step's excitation sample.
template <int GM>
__device__ __forceinline__ void update_groups(const ModeRefs& M, int nc, float e,
                                              const float4 (&F)[GM], int G, int lane,
                                              int* flags) {
  bool bad = false;
#pragma unroll
  for (int g = 0; g < GM; ++g) {
    const int k4 = lane + kWave * g;
    if (g < G && k4 < nc) {
      const int o = 4 * k4;
      float4 xh = ld4(M.xh + o), xl = ld4(M.xl + o);
      float4 dh = ld4(M.dh + o), dl = ld4(M.dl + o);
      const float4 mh = ld4(M.mh + o), ml = ld4(M.ml + o);
      const float4 ph = ld4(M.ph + o), pl = ld4(M.pl + o);
      const float4 rh = ld4(M.rh + o), rl = ld4(M.rl + o);
      const float4 b = ld4(M.b + o);
      const float4 f = F[g];
      ff_step(xh.x, xl.x, dh.x, dl.x, mh.x, ml.x, ph.x, pl.x, rh.x, rl.x, fmaf(b.x, e, -f.x));
      ff_step(xh.y, xl.y, dh.y, dl.y, mh.y, ml.y, ph.y, pl.y, rh.y, rl.y, fmaf(b.y, e, -f.y));
      ff_step(xh.z, xl.z, dh.z, dl.z, mh.z, ml.z, ph.z, pl.z, rh.z, rl.z, fmaf(b.z, e, -f.z));
      ff_step(xh.w, xl.w, dh.w, dl.w, mh.w, ml.w, ph.w, pl.w, rh.w, rl.w, fmaf(b.w, e, -f.w));
      bad |= !(isfinite(xh.x) && isfinite(xh.y) && isfinite(xh.z) && isfinite(xh.w));
      st4(M.xh + o, xh);
      st4(M.xl + o, xl);
      st4(M.dh + o, dh);
      st4(M.dl + o, dl);
    }
  }
  if (__any(bad) && lane == 0) atomicOr(&flags[1], 1);
}

// GM: float4 column groups per lane the launch supports (modes <= 256 GM).
// NW: waves per workgroup.  A unit's rows are divided among the NW waves,
// each sweeping its share with its own LDS reduction region; the per-wave
// partial forces are summed through those regions by wave 0, which also owns
// the output, the exchange with other workgroups and the state update.
// RES: each workgroup owns exactly one unit, whose state and coefficients
// wave 0 copies to LDS before the first step and whose state it writes back
// after the last, so that a step's output, update and recording touch no
// global memory besides the excitation sample and the output (small,
// latency-bound launches, where each global round trip is a large part of a
// step).  Only wave 0 reads or writes these arrays, so they need no barrier.
template <int GM, int NW, bool RES>
__global__ void __launch_bounds__(kWave * NW) step_kernel(StepParams P) {
  extern __shared__ float4 lds4[];
  StepLds L = step_lds(reinterpret_cast<float*>(lds4), NW, P.red_floats);
  float* Xs = L.xs;
  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform by construction; readfirstlane tells the compiler, so that
  // the row ranges and the block walks derived from it stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  float* red = L.red + wave * P.red_floats;
  const int u0 = P.wg_begin[blockIdx.x];
  const int u1 = P.wg_begin[blockIdx.x + 1];
  const long long base = *P.step_base;

  auto refs = [&](const UnitDev& U, const InstDev& I) {
    ModeRefs M;
    if constexpr (RES) {
      float* R = L.res;
      const int S = P.res_stride;
      M.xh = R;
      M.xl = R + S;
      M.dh = R + 2 * S;
      M.dl = R + 3 * S;
      M.mh = R + 4 * S;
      M.ml = R + 5 * S;
      M.ph = R + 6 * S;
      M.pl = R + 7 * S;
      M.rh = R + 8 * S;
      M.rl = R + 9 * S;
      M.b = R + 10 * S;
      M.c = R + 11 * S;
      M.lam = R + 12 * S;
    } else {
      M.xh = P.x_hi + U.state_off;
      M.xl = P.x_lo + U.state_off;
      M.dh = P.d_hi + U.state_off;
      M.dl = P.d_lo + U.state_off;
      M.mh = P.m_hi + I.mode_off;
      M.ml = P.m_lo + I.mode_off;
      M.ph = P.p_hi + I.mode_off;
      M.pl = P.p_lo + I.mode_off;
      M.rh = P.r_hi + I.mode_off;
      M.rl = P.r_lo + I.mode_off;
      M.b = P.b_ext + I.mode_off;
      M.c = P.c_out + I.mode_off;
      M.lam = P.lam + I.mode_off;
    }
    return M;
  };
  // resident state: copy in before the first step, write back after the last
  // (or when a barrier gives up); the host sizes res_stride >= ntp
  auto res_copy = [&](bool in) {
    if (!RES || wave != 0 || u1 <= u0) return;
    const UnitDev U = P.unit[u0];
    const InstDev I = P.inst[U.inst];
    const int nc = I.ntp >> 2;
    float* R = L.res;
    const int S = P.res_stride;
    float* gs[4] = {P.x_hi + U.state_off, P.x_lo + U.state_off, P.d_hi + U.state_off,
                    P.d_lo + U.state_off};
    const float* gc[9] = {P.m_hi, P.m_lo, P.p_hi, P.p_lo, P.r_hi, P.r_lo, P.b_ext, P.c_out, P.lam};
    for (int k4 = lane; k4 < nc; k4 += kWave) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (in)
          st4(R + a * S + 4 * k4, ld4(gs[a] + 4 * k4));
        else
          st4(gs[a] + 4 * k4, ld4(R + a * S + 4 * k4));
      }
      if (in) {
#pragma unroll
        for (int a = 0; a < 9; ++a) st4(R + (4 + a) * S + 4 * k4, ld4(gc[a] + I.mode_off + 4 * k4));
      }
    }
  };
  res_copy(true);

  for (int s = 0; s < P.n_steps; ++s) {
    const long long n = base + s;
    // ---------------- phase 1: output, force, and update of whole units
    for (int u = u0; u < u1; ++u) {
      const UnitDev U = P.unit[u];
      const InstDev I = P.inst[U.inst];
      const ModeRefs M = refs(U, I);
      const int nc = I.ntp >> 2;
      const int G = (nc + kWave - 1) / kWave;
      float spart = 0.f;
      // the excitation sample is fetched first so that its latency overlaps
      // the force evaluation
      float e = 0.f;
      if (wave == 0 && n < I.n_exc) e = P.e_ext[I.e_off + n];
      if (wave == 0) {
        float ypart = 0.f;
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) {
            const float4 xh = ld4(M.xh + 4 * k4);
            const float4 c = ld4(M.c + 4 * k4);
            ypart += dot4(c, xh);
            if (I.kind == KIND_VK) {
              st4(Xs + 4 * k4, xh);
            } else if (I.kind == KIND_TENSION) {
              const float4 l = ld4(M.lam + 4 * k4);
              const float4 lx = make_float4(l.x * xh.x, l.y * xh.y, l.z * xh.z, l.w * xh.w);
              spart += dot4(lx, xh);
            }
          }
        }
        if (U.slab == 0) {
          const float yv = wave_sum(ypart);
          if (lane == 0 && P.y) P.y[(long long)I.out_row * P.y_stride + s] = yv;
          if (P.ckpt && n % P.ckpt_every == 0) {
            float* cp = P.ckpt + (n / P.ckpt_every) * 4LL * P.mode_floats + I.mode_off;
            for (int g = 0; g < GM; ++g) {
              const int k4 = lane + kWave * g;
              if (g < G && k4 < nc) {
                st4(cp + 4 * k4, ld4(M.xh + 4 * k4));
                st4(cp + P.mode_floats + 4 * k4, ld4(M.xl + 4 * k4));
                st4(cp + 2 * P.mode_floats + 4 * k4, ld4(M.dh + 4 * k4));
                st4(cp + 3 * P.mode_floats + 4 * k4, ld4(M.dl + 4 * k4));
              }
            }
          }
          if (P.rec_x) {
            const long long ro = (n - P.rec_base) * P.mode_floats + I.mode_off;
            for (int g = 0; g < GM; ++g) {
              const int k4 = lane + kWave * g;
              if (g < G && k4 < nc) {
                st4(P.rec_x + ro + 4 * k4, ld4(M.xh + 4 * k4));
                st4(P.rec_d + ro + 4 * k4, ld4(M.dh + 4 * k4));
              }
            }
          }
        }
      }
      float4 Fa[GM];
#pragma unroll
      for (int g = 0; g < GM; ++g) Fa[g] = f4(0.f);
      if (I.kind == KIND_VK) {
        __syncthreads();  // q^n in LDS
        const int R = U.row1 - U.row0;
        if (RES && NW > 1 && !I.blk && 2 * R <= NW) {
          // one unit per workgroup with at most half as many rows as waves:
          // the waves share its row blocks evenly (with whole rows per wave
          // otherwise, measured faster there: 50/50 plates 9.1 us per step
          // against 11.8, 100/100 in 7-row slabs 11.7 against 14.6)
          const int nblk = (I.nt + U.qs - 1) / U.qs;
          const int T = R * nblk;
          float* xv = L.xch;
          int* xr = reinterpret_cast<int*>(L.xch + 2 * NW);
          float* defer = red + 2 * U.qs * I.ntp;
          vk_rows_range<GM, (NW == 8 && GM <= 2) ? 3 : 2, kKeep>(
              P.H + I.h_off, I.nt, I.ntp, U.qs, U.row0, (T * wave) / NW, (T * (wave + 1)) / NW, Xs, red, Fa, G,
              lane, defer, xv + 2 * wave, xr + 2 * wave);
          bool cut = false;  // a wave boundary inside a row
          for (int w = 1; w < NW; ++w) cut |= ((T * w) / NW) % nblk != 0;
          if (cut) {
            __syncthreads();  // every wave's partial eta_n of the rows it shares
            vk_rows_finish<GM>(xv, xr, NW, wave, I.ntp, defer, Fa, G, lane);
          }
        } else {
          const int r0 = U.row0 + (R * wave) / NW, r1 = U.row0 + (R * (wave + 1)) / NW;
          if (I.blk)
            vk_rows_blk<GM>(P.H + I.h_off, P.jmap + I.jmap_off, I, r0, r1, Xs, red, Fa, G, lane);
          else
            vk_rows<GM, (NW == 8 && GM <= 2) ? 3 : 2, RES ? kKeep : kStream>(
                P.H + I.h_off, I.nt, I.ntp, U.qs, r0, r1, Xs, red, Fa, G, lane);
        }
        if (NW > 1) {
#pragma unroll
          for (int g = 0; g < GM; ++g) {
            const int k4 = lane + kWave * g;
            if (g < G && k4 < nc) st4(red + 4 * k4, Fa[g]);
          }
          __syncthreads();
          if (wave == 0) {
#pragma unroll
            for (int g = 0; g < GM; ++g) {
              const int k4 = lane + kWave * g;
              if (g < G && k4 < nc)
                for (int w = 1; w < NW; ++w) Fa[g] = add4(Fa[g], ld4(L.red + w * P.red_floats + 4 * k4));
            }
          }
        }
      } else if (I.kind == KIND_TENSION && wave == 0) {
        const float S = wave_sum(spart) * I.kappa;
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) {
            const float4 xh = ld4(M.xh + 4 * k4);
            const float4 l = ld4(M.lam + 4 * k4);
            Fa[g] = make_float4(l.x * xh.x * S, l.y * xh.y * S, l.z * xh.z * S, l.w * xh.w * S);
          }
        }
      }
      if (wave == 0) {
        if (I.nslab == 1) {
          update_groups<GM>(M, nc, e, Fa, G, lane, P.flags);
        } else {
          // this instance's exchange region: [2][nslab][ntp] floats
          const v4i pr = buf_rsrc(P.part + I.part_off, 8 * I.nslab * I.ntp);
          const int dst = 4 * ((int)(n & 1) * I.nslab + U.slab) * I.ntp;
#pragma unroll
          for (int g = 0; g < GM; ++g) {
            const int k4 = lane + kWave * g;
            if (g < G && k4 < nc) st4_coherent(pr, dst + 16 * k4, Fa[g]);
          }
          publish_fence();
          __builtin_amdgcn_wave_barrier();
          if (lane == 0)
            __hip_atomic_store(&P.ctr[I.ctr_off + U.slab], (unsigned int)(n + 1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __syncthreads();  // LDS reused by the next unit
    }
    // ---------------- phase 2: split instances wait, sum partials, update
    for (int u = u0; u < u1; ++u) {
      const UnitDev U = P.unit[u];
      const InstDev I = P.inst[U.inst];
      if (I.nslab == 1) continue;
      if (wave == 0) {
        const bool ok = wait_slabs(P.ctr + I.ctr_off, I.nslab, (unsigned int)(n + 1), P.flags, P.timeout_ticks);
        if (lane == 0) L.flag[0] = ok ? 1 : 0;
      }
      __syncthreads();
      if (L.flag[0] == 0) {  // every wave leaves together
        res_copy(false);
        return;
      }
      const int nc = I.ntp >> 2;
      const int G = (nc + kWave - 1) / kWave;
      const v4i pr = buf_rsrc(P.part + I.part_off, 8 * I.nslab * I.ntp);
      const int src = 4 * (int)(n & 1) * I.nslab * I.ntp;  // byte offset of this step's partials
      if (RES && NW > 1 && I.nslab >= 2 * NW) {
        // one unit per workgroup and many slabs: every wave sums every NW-th
        // partial force, and wave 0 adds the waves' sums
        consume_fence();
        float4 F[GM];
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          F[g] = f4(0.f);
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) {
            F[g] = sum_slabs4_coherent(pr, src + 16 * k4, wave, NW, I.nslab, 4 * I.ntp);
            st4(red + 4 * k4, F[g]);
          }
        }
        __syncthreads();
        if (wave == 0) {
          const ModeRefs M = refs(U, I);
          float e = 0.f;
          if (n < I.n_exc) e = P.e_ext[I.e_off + n];
#pragma unroll
          for (int g = 0; g < GM; ++g) {
            const int k4 = lane + kWave * g;
            if (g < G && k4 < nc)
              for (int w = 1; w < NW; ++w) F[g] = add4(F[g], ld4(L.red + w * P.red_floats + 4 * k4));
          }
          update_groups<GM>(M, nc, e, F, G, lane, P.flags);
        }
      } else if (wave == 0) {
        consume_fence();
        const ModeRefs M = refs(U, I);
        float e = 0.f;
        if (n < I.n_exc) e = P.e_ext[I.e_off + n];
        float4 F[GM];
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          F[g] = f4(0.f);
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc)
            for (int t = 0; t < I.nslab; ++t)
              F[g] = add4(F[g], ld4_coherent(pr, src + 4 * t * I.ntp + 16 * k4));
        }
        update_groups<GM>(M, nc, e, F, G, lane, P.flags);
      }
      __syncthreads();  // flag reused
    }
  }
  res_copy(false);
}

__global__ void advance_kernel(long long* step_base, int n_steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_base += n_steps;
}

// Arrival words as they stand after *step_base steps from a reset: every
// slab has published every step (mod 2^32, like the waits' targets).  Lets
// a launch run on words that another context left behind.
__global__ void ctr_fill_kernel(const InstDev* inst, int batch, const long long* step_base,
                                unsigned int* ctr) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const unsigned int v = (unsigned int)(unsigned long long)*step_base;
  for (int t = 0; t < inst[b].nslab; ++t) ctr[inst[b].ctr_off + t] = v;
}

// Symmetry and finiteness of each instance's Ht: out[2b] = max |H - H^T|,
// out[2b+1] = max |H|, both as float bits (non-negative floats order like
// their bit patterns); a non-finite entry reports +inf in both.
__global__ void check_kernel(const float* H, const InstDev* inst, int* out) {
  const InstDev I = inst[blockIdx.y];
  if (I.kind != KIND_VK || I.blk) return;  // blocked tensors are checked on the host
  const long long total = (long long)I.nin * I.nt * I.nt;
  float dmax = 0.f, hmax = 0.f;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % I.nt);
    const long long r = e / I.nt;
    const int k = (int)(r % I.nt);
    const long long n = r / I.nt;
    const float* Hn = H + I.h_off + n * (long long)I.nt * I.ntp;
    const float a = Hn[(long long)k * I.ntp + j];
    const float b = Hn[(long long)j * I.ntp + k];
    if (!isfinite(a)) {
      dmax = INFINITY;
      hmax = INFINITY;
    } else {
      dmax = fmaxf(dmax, fabsf(a - b));
      hmax = fmaxf(hmax, fabsf(a));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmaxf(dmax, __shfl_xor(dmax, o, kWave));
    hmax = fmaxf(hmax, __shfl_xor(hmax, o, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(&out[2 * blockIdx.y], __float_as_int(dmax));
    atomicMax(&out[2 * blockIdx.y + 1], __float_as_int(hmax));
  }
}

}  // namespace modal

// Launch wrappers used by the host code (same translation unit keeps the
// kernels' symbols local to this file).
namespace modal {
// gm: float4 column groups per lane needed by the widest instance (1, 2 or
// 4); nw: waves per workgroup (1, 4 or 8); P.res_stride > 0 selects the
// variant with LDS-resident state (four or eight waves, one unit per
// workgroup).
hipError_t launch_step(const StepParams& P, int gm, int nw, int n_wg, size_t lds_bytes, hipStream_t s) {
#define SL(G, W, R) hipLaunchKernelGGL((step_kernel<G, W, R>), dim3(n_wg), dim3(kWave * W), lds_bytes, s, P)
  if (P.res_stride > 0) {
    if (nw == 8) {
      if (gm <= 1) SL(1, 8, true); else if (gm <= 2) SL(2, 8, true); else SL(4, 8, true);
    } else if (nw == 4) {
      if (gm <= 1) SL(1, 4, true); else if (gm <= 2) SL(2, 4, true); else SL(4, 4, true);
    } else {
      return hipErrorInvalidValue;  // resident launches use four or eight waves
    }
  } else if (nw == 1) {
    if (gm <= 1) SL(1, 1, false); else if (gm <= 2) SL(2, 1, false); else SL(4, 1, false);
  } else if (nw == 8) {
    if (gm <= 1) SL(1, 8, false); else if (gm <= 2) SL(2, 8, false); else SL(4, 8, false);
  } else {
    if (gm <= 1) SL(1, 4, false); else if (gm <= 2) SL(2, 4, false); else SL(4, 4, false);
  }
#undef SL
  return hipGetLastError();
}
hipError_t launch_advance(long long* step_base, int n, hipStream_t s) {
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step_base, n);
  return hipGetLastError();
}
hipError_t launch_ctr_fill(const InstDev* inst, int batch, const long long* step_base, unsigned int* ctr,
                           hipStream_t s) {
  hipLaunchKernelGGL(ctr_fill_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, inst, batch, step_base, ctr);
  return hipGetLastError();
}
hipError_t launch_check(const float* H, const InstDev* inst, int batch, int* out, hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(64, batch), dim3(256), 0, s, H, inst, out);
  return hipGetLastError();
}
hipError_t step_occupancy(int* blocks_per_cu, int gm, int nw, size_t lds_bytes, bool res) {
#define SO(G, W, R) \
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, step_kernel<G, W, R>, kWave * W, lds_bytes)
  if (res) {
    if (nw == 8) {
      if (gm <= 1) SO(1, 8, true);
      if (gm <= 2) SO(2, 8, true);
      SO(4, 8, true);
    }
    if (nw == 4) {
      if (gm <= 1) SO(1, 4, true);
      if (gm <= 2) SO(2, 4, true);
      SO(4, 4, true);
    }
    *blocks_per_cu = 0;
    return hipSuccess;
  }
  if (nw == 1) {
    if (gm <= 1) SO(1, 1, false);
    if (gm <= 2) SO(2, 1, false);
    SO(4, 1, false);
  }
  if (nw == 8) {
    if (gm <= 1) SO(1, 8, false);
    if (gm <= 2) SO(2, 8, false);
    SO(4, 8, false);
  }
  if (gm <= 1) SO(1, 4, false);
  if (gm <= 2) SO(2, 4, false);
  SO(4, 4, false);
#undef SO
}
}  // namespace modal
