// Reverse (adjoint) sweep of the modal time loop over one recorded segment.
//
// Back-propagation through the increment-form recursion of the step kernel
// (paper: Sec. 4.3 fits by propagating gradients through the integrator):
//   db^{n+1} = qb^{n+1} - p db^{n+2},  u^n = r db^{n+1},
//   qb^n     = ybar^n c + qb^{n+1} + m db^{n+1} - J(q^n) u^n,
// with J = dF/dq symmetric.  For the von Karman force one pass over a row of
// Ht with two right-hand sides gives V = Ht q and W = Ht u, eta = V.q,
// w = V.u and (J u) += 2 w V + eta W, F += eta V.  Per-mode float-float
// accumulators collect dL/dm, dL/dp, dL/dr, dL/dc and the force-scale term
// u.F; an optional tangent tensor Hd adds the directional derivative
// -(Vd.q) (V.u) - eta (Vd.u) per row, Vd = Hd q.  Work partition, slab
// exchange and barriers are those of the forward kernel.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace modal {

template <int GM, bool TAN, int DEPTH, int POL>
__device__ void vk_rows2(const float* __restrict__ Hb, const float* __restrict__ Hdb, int nt,
                         int ntp, int qs, int row0, int row1, const float* Xs, const float* Us,
                         float* red, float4 (&Ju)[GM], float4 (&Fa)[GM], float& tsum, int G,
                         int lane, float* rrow, float* teta, float* tw) {
  // Same sweep as the forward kernel (contiguous blocks of qs stored rows,
  // per-block buffer resources, next block loaded ahead) with two
  // right-hand sides, q and u, and optionally the tangent tensor times q.
  constexpr int J = kSweepLoads;
  constexpr int NR = TAN ? 3 : 2;  // reduced vectors per row: V, W (, Vd)
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
  const int slab = qs * ntp;
  int ln = row0, lb = 0;
  auto load = [&](float4 (&h)[J], float4 (&hd)[J]) {
    const bool live = ln < row1;
    const long long o = live ? (long long)ln * row_floats + (long long)lb * blk_floats : 0;
    const int bytes = live ? (lb == nblk - 1 ? last_bytes : blk_bytes) : 0;
    const v4i r = buf_rsrc(Hb + o, bytes);
#pragma unroll
    for (int j = 0; j < J; ++j) h[j] = buf_ld4<POL>(r, voff[j]);
    if (TAN) {
      const v4i rd = buf_rsrc(Hdb + o, bytes);
#pragma unroll
      for (int j = 0; j < J; ++j) hd[j] = buf_ld4<POL>(rd, voff[j]);
    }
    if (++lb == nblk) {
      lb = 0;
      ++ln;
    }
  };
  float4 ha[J], hb[J], hda[J], hdb[J], aV[J], aW[J], aD[J];
#pragma unroll
  for (int j = 0; j < J; ++j) aV[j] = aW[j] = aD[j] = f4(0.f);
  int n = row0, b = 0;
  auto step = [&](float4 (&hc)[J], float4 (&hdc)[J], float4 (&hn)[J], float4 (&hdn)[J]) -> bool {
    load(hn, hdn);
    const int q0 = b * qs;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int qi = min(q0 + sub[j], nt - 1);
      const float x = Xs[qi], u = Us[qi];
      aV[j] = fma4(hc[j], x, aV[j]);
      aW[j] = fma4(hc[j], u, aW[j]);
      if (TAN) aD[j] = fma4(hdc[j], x, aD[j]);
    }
    if (++b < nblk) return true;
    float* rb = red + (n & 1) * NR * slab;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (voff[j] < blk_bytes) {
        const int o = voff[j] >> 2;
        st4(rb + o, aV[j]);
        st4(rb + slab + o, aW[j]);
        if (TAN) st4(rb + 2 * slab + o, aD[j]);
      }
    }
    wave_lds_sync();
    float eta = 0.f, w = 0.f, etad = 0.f, vdu = 0.f;
    float4 V[GM], W[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      V[g] = W[g] = f4(0.f);
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) {
        const float4 sv = sum_strided4(rb + 4 * k4, qs, ntp);
        const float4 sw = sum_strided4(rb + slab + 4 * k4, qs, ntp);
        const float4 sd = TAN ? sum_strided4(rb + 2 * slab + 4 * k4, qs, ntp) : f4(0.f);
        V[g] = sv;
        W[g] = sw;
        const float4 x = ld4(Xs + 4 * k4), u = ld4(Us + 4 * k4);
        eta += dot4(sv, x);
        w += dot4(sv, u);
        if (TAN) {
          etad += dot4(sd, x);
          vdu += dot4(sd, u);
        }
      }
    }
    eta = wave_sum(eta);
    w = wave_sum(w);
    // row-scale gradient term of this step (summed over steps afterwards)
    if (rrow && lane == 0) rrow[n] = -2.f * eta * w;
    // eta_n and V_n . u of this step for the full tensor gradient
    if (teta && lane == 0) {
      teta[n] = eta;
      tw[n] = w;
    }
    if (TAN) {
      etad = wave_sum(etad);
      vdu = wave_sum(vdu);
      tsum -= etad * w + eta * vdu;
    }
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      Ju[g] = fma4(V[g], 2.f * w, fma4(W[g], eta, Ju[g]));
      Fa[g] = fma4(V[g], eta, Fa[g]);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) aV[j] = aW[j] = aD[j] = f4(0.f);
    b = 0;
    return ++n < row1;
  };
  load(ha, hda);
  if (DEPTH == 2) {
    while (step(ha, hda, hb, hdb) && step(hb, hdb, ha, hda)) {
    }
  } else {  // three buffers: two blocks' loads in flight
    float4 hx[J], hdx[J];
    load(hb, hdb);
    while (step(ha, hda, hx, hdx) && step(hb, hdb, ha, hda) && step(hx, hdx, hb, hdb)) {
    }
  }
}

// vk_rows2 over a range of row blocks [t0, t1) of the unit whose rows start
// at row0 (block t is block t % nblk of row row0 + t / nblk), for one-unit
// workgroups whose waves share the unit's blocks evenly.  Rows wholly in the
// range are finished here.  For a row the range cuts, the partial V, W (and
// Vd) are parked in `defer` (slot s at s NR ntp) and the partial eta, V.u,
// Vd.q and Vd.u with the row index in the wave's exchange words (slot 0: a
// row entered mid-row, slot 1: a row left mid-row), for vk_rows2_finish.
template <int GM, bool TAN, int DEPTH, int POL>
__device__ void vk_rows2_range(const float* __restrict__ Hb, const float* __restrict__ Hdb, int nt,
                               int ntp, int qs, int row0, int t0, int t1, const float* Xs,
                               const float* Us, float* red, float4 (&Ju)[GM], float4 (&Fa)[GM],
                               float& tsum, int G, int lane, float* rrow, float* teta, float* tw,
                               float* defer, float* xv, int* xr) {
  constexpr int J = kSweepLoads;
  constexpr int NR = TAN ? 3 : 2;
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
  const int slab = qs * ntp;
  int lt = t0, ln = row0 + t0 / nblk, lb = t0 % nblk;
  auto load = [&](float4 (&h)[J], float4 (&hd)[J]) {
    const bool live = lt < t1;
    const long long o = live ? (long long)ln * row_floats + (long long)lb * blk_floats : 0;
    const int bytes = live ? (lb == nblk - 1 ? last_bytes : blk_bytes) : 0;
    const v4i r = buf_rsrc(Hb + o, bytes);
#pragma unroll
    for (int j = 0; j < J; ++j) h[j] = buf_ld4<POL>(r, voff[j]);
    if (TAN) {
      const v4i rd = buf_rsrc(Hdb + o, bytes);
#pragma unroll
      for (int j = 0; j < J; ++j) hd[j] = buf_ld4<POL>(rd, voff[j]);
    }
    ++lt;
    if (++lb == nblk) {
      lb = 0;
      ++ln;
    }
  };
  float4 ha[J], hb[J], hda[J], hdb[J], aV[J], aW[J], aD[J];
#pragma unroll
  for (int j = 0; j < J; ++j) aV[j] = aW[j] = aD[j] = f4(0.f);
  int t = t0, n = row0 + t0 / nblk, b = t0 % nblk, bfirst = b;
  auto step = [&](float4 (&hc)[J], float4 (&hdc)[J], float4 (&hn)[J], float4 (&hdn)[J]) -> bool {
    load(hn, hdn);
    const int q0 = b * qs;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int qi = min(q0 + sub[j], nt - 1);
      const float x = Xs[qi], u = Us[qi];
      aV[j] = fma4(hc[j], x, aV[j]);
      aW[j] = fma4(hc[j], u, aW[j]);
      if (TAN) aD[j] = fma4(hdc[j], x, aD[j]);
    }
    ++t;
    if (++b < nblk && t < t1) return true;
    float* rb = red + (n & 1) * NR * slab;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (voff[j] < blk_bytes) {
        const int o = voff[j] >> 2;
        st4(rb + o, aV[j]);
        st4(rb + slab + o, aW[j]);
        if (TAN) st4(rb + 2 * slab + o, aD[j]);
      }
    }
    wave_lds_sync();
    float eta = 0.f, w = 0.f, etad = 0.f, vdu = 0.f;
    float4 V[GM], W[GM], D[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      V[g] = W[g] = D[g] = f4(0.f);
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) {
        const float4 sv = sum_strided4(rb + 4 * k4, qs, ntp);
        const float4 sw = sum_strided4(rb + slab + 4 * k4, qs, ntp);
        const float4 sd = TAN ? sum_strided4(rb + 2 * slab + 4 * k4, qs, ntp) : f4(0.f);
        V[g] = sv;
        W[g] = sw;
        D[g] = sd;
        const float4 x = ld4(Xs + 4 * k4), u = ld4(Us + 4 * k4);
        eta += dot4(sv, x);
        w += dot4(sv, u);
        if (TAN) {
          etad += dot4(sd, x);
          vdu += dot4(sd, u);
        }
      }
    }
    eta = wave_sum(eta);
    w = wave_sum(w);
    if (TAN) {
      etad = wave_sum(etad);
      vdu = wave_sum(vdu);
    }
    if (bfirst == 0 && b == nblk) {
      if (rrow && lane == 0) rrow[n] = -2.f * eta * w;
      if (teta && lane == 0) {
        teta[n] = eta;
        tw[n] = w;
      }
      if (TAN) tsum -= etad * w + eta * vdu;
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        Ju[g] = fma4(V[g], 2.f * w, fma4(W[g], eta, Ju[g]));
        Fa[g] = fma4(V[g], eta, Fa[g]);
      }
    } else {
      const int slot = bfirst > 0 ? 0 : 1;
      float* dp = defer + slot * NR * ntp;
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        const int k4 = lane + kWave * g;
        if (g < G && k4 < nc) {
          st4(dp + 4 * k4, V[g]);
          st4(dp + ntp + 4 * k4, W[g]);
          if (TAN) st4(dp + 2 * ntp + 4 * k4, D[g]);
        }
      }
      if (lane == 0) {
        xv[slot * kXchVals] = eta;
        xv[slot * kXchVals + 1] = w;
        xv[slot * kXchVals + 2] = etad;
        xv[slot * kXchVals + 3] = vdu;
        xr[slot] = n;
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) aV[j] = aW[j] = aD[j] = f4(0.f);
    b = 0;
    bfirst = 0;
    ++n;
    return t < t1;
  };
  load(ha, hda);
  if (DEPTH == 2) {
    while (step(ha, hda, hb, hdb) && step(hb, hdb, ha, hda)) {
    }
  } else {
    float4 hx[J], hdx[J];
    load(hb, hdb);
    while (step(ha, hda, hx, hdx) && step(hb, hdb, ha, hda) && step(hx, hdx, hb, hdb)) {
    }
  }
}

// Completes the rows vk_rows2_range left to several waves, after a workgroup
// barrier: the row's eta, V.u, Vd.q and Vd.u are the sums of every sharing
// wave's partials (in wave order); each sharing wave adds its partial vectors
// times them, and the wave that holds the row's first block (slot 1) writes
// the row's records and its tangent term.  xv, xr: exchange words of all nw
// waves (this wave's at 2 wave).
template <int GM, bool TAN>
__device__ void vk_rows2_finish(const float* xv, const int* xr, int nw, int wave, int ntp,
                                const float* defer, float4 (&Ju)[GM], float4 (&Fa)[GM], float& tsum,
                                int G, int lane, float* rrow, float* teta, float* tw) {
  constexpr int NR = TAN ? 3 : 2;
  const int nc = ntp >> 2;
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int n = xr[2 * wave + slot];
    if (n < 0) continue;
    float eta = 0.f, w = 0.f, etad = 0.f, vdu = 0.f;
    for (int i = 0; i < 2 * nw; ++i)
      if (xr[i] == n) {
        eta += xv[i * kXchVals];
        w += xv[i * kXchVals + 1];
        etad += xv[i * kXchVals + 2];
        vdu += xv[i * kXchVals + 3];
      }
    const float* dp = defer + slot * NR * ntp;
#pragma unroll
    for (int g = 0; g < GM; ++g) {
      const int k4 = lane + kWave * g;
      if (g < G && k4 < nc) {
        const float4 V = ld4(dp + 4 * k4), W = ld4(dp + ntp + 4 * k4);
        Ju[g] = fma4(V, 2.f * w, fma4(W, eta, Ju[g]));
        Fa[g] = fma4(V, eta, Fa[g]);
      }
    }
    if (slot == 1) {
      if (rrow && lane == 0) rrow[n] = -2.f * eta * w;
      if (teta && lane == 0) {
        teta[n] = eta;
        tw[n] = w;
      }
      if (TAN) tsum -= etad * w + eta * vdu;
    }
  }
}

__device__ __forceinline__ void acc_add(float* acc, int k, int sf, int i, ff v) {
  ff a{acc[(2 * k) * (long long)sf + i], acc[(2 * k + 1) * (long long)sf + i]};
  a = ff_add(a, v);
  acc[(2 * k) * (long long)sf + i] = a.hi;
  acc[(2 * k + 1) * (long long)sf + i] = a.lo;
}

// u^n = r db^{n+1}, db^{n+1} = qb^{n+1} - p db^{n+2}, of four consecutive
// modes from the adjoint state (the high parts of u).
__device__ __forceinline__ float4 adj_u4(const GradParams& P, int so, int mo) {
  const float4 qh4 = ld4(P.qb_hi + so), ql4 = ld4(P.qb_lo + so);
  const float4 dh4 = ld4(P.db_hi + so), dl4 = ld4(P.db_lo + so);
  const float4 ph4 = ld4(P.p_hi + mo), pl4 = ld4(P.p_lo + mo);
  const float4 rh4 = ld4(P.r_hi + mo), rl4 = ld4(P.r_lo + mo);
  const float qh[4] = {qh4.x, qh4.y, qh4.z, qh4.w}, ql[4] = {ql4.x, ql4.y, ql4.z, ql4.w};
  const float dh[4] = {dh4.x, dh4.y, dh4.z, dh4.w}, dl[4] = {dl4.x, dl4.y, dl4.z, dl4.w};
  const float ph[4] = {ph4.x, ph4.y, ph4.z, ph4.w}, pl[4] = {pl4.x, pl4.y, pl4.z, pl4.w};
  const float rh[4] = {rh4.x, rh4.y, rh4.z, rh4.w}, rl[4] = {rl4.x, rl4.y, rl4.z, rl4.w};
  float us[4];
#pragma unroll
  for (int e4 = 0; e4 < 4; ++e4) {
    const ff t = ff_mul({ph[e4], pl[e4]}, {dh[e4], dl[e4]});
    const ff db = ff_add({qh[e4], ql[e4]}, {-t.hi, -t.lo});
    us[e4] = ff_mul({rh[e4], rl[e4]}, db).hi;
  }
  return make_float4(us[0], us[1], us[2], us[3]);
}

// Finishes step n for the modes of one unit given the full J u and F.  The
// adjoint state, coefficients and accumulators of a lane's four modes move
// as float4 (per-unit state and per-mode arrays start on multiples of 4).
template <int GM>
__device__ void adj_post(const GradParams& P, const InstDev& I, const UnitDev& U, long long n,
                         const float4 (&Ju)[GM], const float4 (&F)[GM], int G, int lane) {
  const int nc = I.ntp >> 2;
  const float e = n < I.n_exc ? P.e_ext[I.e_off + n] : 0.f;
  const float yb = P.ybar[(long long)I.out_row * P.ybar_stride + n];
  const long long ro = (n - P.seg_base) * P.mode_floats + I.mode_off;
  const long long sf = P.state_floats;
  const bool accumulate = U.slab == 0;
#pragma unroll
  for (int g = 0; g < GM; ++g) {
    const int k4 = lane + kWave * g;
    if (!(g < G && k4 < nc)) continue;
    const int so = U.state_off + 4 * k4;
    const int mo = I.mode_off + 4 * k4;
    const float4 x4 = ld4(P.rec_x + ro + 4 * k4), d4 = ld4(P.rec_d + ro + 4 * k4);
    const float4 b4 = ld4(P.b_ext + mo), c4 = ld4(P.c_out + mo);
    const float4 qh4 = ld4(P.qb_hi + so), ql4 = ld4(P.qb_lo + so);
    const float4 dh4 = ld4(P.db_hi + so), dl4 = ld4(P.db_lo + so);
    const float4 ph4 = ld4(P.p_hi + mo), pl4 = ld4(P.p_lo + mo);
    const float4 rh4 = ld4(P.r_hi + mo), rl4 = ld4(P.r_lo + mo);
    const float4 mh4 = ld4(P.m_hi + mo), ml4 = ld4(P.m_lo + mo);
    float4 ah[5], al[5];
    if (accumulate) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        ah[k] = ld4(P.acc + (2 * k) * sf + so);
        al[k] = ld4(P.acc + (2 * k + 1) * sf + so);
      }
    }
    const float xs[4] = {x4.x, x4.y, x4.z, x4.w}, ds[4] = {d4.x, d4.y, d4.z, d4.w};
    const float bs[4] = {b4.x, b4.y, b4.z, b4.w}, cs[4] = {c4.x, c4.y, c4.z, c4.w};
    const float js[4] = {Ju[g].x, Ju[g].y, Ju[g].z, Ju[g].w};
    const float fs[4] = {F[g].x, F[g].y, F[g].z, F[g].w};
    const float qh[4] = {qh4.x, qh4.y, qh4.z, qh4.w}, ql[4] = {ql4.x, ql4.y, ql4.z, ql4.w};
    const float dh[4] = {dh4.x, dh4.y, dh4.z, dh4.w}, dl[4] = {dl4.x, dl4.y, dl4.z, dl4.w};
    const float phs[4] = {ph4.x, ph4.y, ph4.z, ph4.w}, pls[4] = {pl4.x, pl4.y, pl4.z, pl4.w};
    const float rhs[4] = {rh4.x, rh4.y, rh4.z, rh4.w}, rls[4] = {rl4.x, rl4.y, rl4.z, rl4.w};
    const float mhs[4] = {mh4.x, mh4.y, mh4.z, mh4.w}, mls[4] = {ml4.x, ml4.y, ml4.z, ml4.w};
    float ahs[5][4], als[5][4];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      ahs[k][0] = ah[k].x; ahs[k][1] = ah[k].y; ahs[k][2] = ah[k].z; ahs[k][3] = ah[k].w;
      als[k][0] = al[k].x; als[k][1] = al[k].y; als[k][2] = al[k].z; als[k][3] = al[k].w;
    }
    float oqh[4], oql[4], odh[4], odl[4];
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
      // db^{n+1} = qb^{n+1} - p db^{n+2},  u^n = r db^{n+1}
      const ff t = ff_mul({phs[e4], pls[e4]}, {dh[e4], dl[e4]});
      const ff db = ff_add({qh[e4], ql[e4]}, {-t.hi, -t.lo});
      const ff u = ff_mul({rhs[e4], rls[e4]}, db);
      if (accumulate) {
        const ff v[5] = {ff_mul_f(db, xs[e4]), ff_mul_f(db, -ds[e4]), ff_mul_f(db, fmaf(bs[e4], e, -fs[e4])),
                         two_prod(yb, xs[e4]), ff_mul_f(u, -fs[e4])};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const ff a = ff_add({ahs[k][e4], als[k][e4]}, v[k]);
          ahs[k][e4] = a.hi;
          als[k][e4] = a.lo;
        }
      }
      // qb^n = ybar c + qb^{n+1} + m db^{n+1} - (J u)
      ff qb = {qh[e4], ql[e4]};
      qb = ff_add(qb, ff_mul({mhs[e4], mls[e4]}, db));
      qb = ff_add(qb, two_prod(yb, cs[e4]));
      qb = ff_add(qb, {-js[e4], 0.f});
      oqh[e4] = qb.hi;
      oql[e4] = qb.lo;
      odh[e4] = db.hi;
      odl[e4] = db.lo;
    }
    if (accumulate) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        st4(P.acc + (2 * k) * sf + so, make_float4(ahs[k][0], ahs[k][1], ahs[k][2], ahs[k][3]));
        st4(P.acc + (2 * k + 1) * sf + so, make_float4(als[k][0], als[k][1], als[k][2], als[k][3]));
      }
    }
    st4(P.qb_hi + so, make_float4(oqh[0], oqh[1], oqh[2], oqh[3]));
    st4(P.qb_lo + so, make_float4(oql[0], oql[1], oql[2], oql[3]));
    st4(P.db_hi + so, make_float4(odh[0], odh[1], odh[2], odh[3]));
    st4(P.db_lo + so, make_float4(odl[0], odl[1], odl[2], odl[3]));
  }
}

// GM: float4 column groups per lane; TAN: tangent tensor present; NW: waves
// per workgroup.  As in the forward kernel, the waves of a workgroup divide a
// unit's rows among themselves and wave 0 sums their partial J u, F and
// tangent sums, finishes the step or publishes the unit's share.
template <int GM, bool TAN, int NW, bool SPLIT>
__global__ void __launch_bounds__(kWave * NW) grad_kernel(GradParams P) {
  extern __shared__ float4 lds4[];
  const GradLds L = grad_lds(reinterpret_cast<float*>(lds4));
  float* Xs = L.xs;
  float* Us = L.us;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  float* red = L.red + wave * P.red_floats;
  const int u0 = P.wg_begin[blockIdx.x];
  const int u1 = P.wg_begin[blockIdx.x + 1];

  for (int s = 0; s < P.seg_len; ++s) {
    const long long n = P.seg_base + P.seg_len - 1 - s;  // absolute step, descending
    const long long rstep = P.done_before + s;          // reverse steps done so far
    for (int u = u0; u < u1; ++u) {
      const UnitDev U = P.unit[u];
      const InstDev I = P.inst[U.inst];
      const int nc = I.ntp >> 2;
      const int G = (nc + kWave - 1) / kWave;
      const long long ro = (n - P.seg_base) * P.mode_floats + I.mode_off;
      float tsum = 0.f, sx = 0.f, sxu = 0.f;
      float4 Ju[GM], Fa[GM];
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        Ju[g] = Fa[g] = f4(0.f);
        const int k4 = lane + kWave * g;
        if (wave == 0 && g < G && k4 < nc) {
          const float4 x4 = ld4(P.rec_x + ro + 4 * k4);
          const float4 u4 = adj_u4(P, U.state_off + 4 * k4, I.mode_off + 4 * k4);
          if (I.kind == KIND_VK) {
            st4(Xs + 4 * k4, x4);
            st4(Us + 4 * k4, u4);
            if (P.urec && U.slab == 0) st4(P.urec + ro + 4 * k4, u4);
          } else if (I.kind == KIND_TENSION) {
            const float4 l = ld4(P.lam + I.mode_off + 4 * k4);
            const float4 lx = make_float4(l.x * x4.x, l.y * x4.y, l.z * x4.z, l.w * x4.w);
            sx += dot4(lx, x4);
            sxu += dot4(lx, u4);
            Ju[g] = u4;  // temporarily holds u
          }
        }
      }
      if (I.kind == KIND_VK) {
        __syncthreads();  // q^n, u^n in LDS
        const int R = U.row1 - U.row0;
        const int r0 = U.row0 + (R * wave) / NW, r1 = U.row0 + (R * (wave + 1)) / NW;
        float* rrow = P.rrec ? P.rrec + (long long)s * P.rows_total + I.row_off : nullptr;
        float* teta = P.trec ? P.trec + (n - P.seg_base) * 2LL * P.rows_total + I.row_off : nullptr;
        float* tw = teta ? teta + P.rows_total : nullptr;
        if (SPLIT && NW > 1 && 2 * R <= NW) {
          // one unit per workgroup with at most half as many rows as waves:
          // the waves share its row blocks evenly
          const int nblk = (I.nt + U.qs - 1) / U.qs;
          const int T = R * nblk;
          constexpr int NR = TAN ? 3 : 2;
          float* xv = L.xch;
          int* xr = reinterpret_cast<int*>(L.xch + 2 * NW * kXchVals);
          float* defer = red + 2 * NR * U.qs * I.ntp;
          vk_rows2_range<GM, TAN, (NW == 8 && GM <= 2) ? 3 : 2, kKeep>(
              P.H + I.h_off, TAN ? P.Hd + I.h_off : nullptr, I.nt, I.ntp, U.qs, U.row0, (T * wave) / NW,
              (T * (wave + 1)) / NW, Xs, Us, red, Ju, Fa, tsum, G, lane, rrow, teta, tw, defer,
              xv + 2 * wave * kXchVals, xr + 2 * wave);
          bool cut = false;  // a wave boundary inside a row
          for (int w = 1; w < NW; ++w) cut |= ((T * w) / NW) % nblk != 0;
          if (cut) {
            __syncthreads();  // every wave's partials of the rows it shares
            vk_rows2_finish<GM, TAN>(xv, xr, NW, wave, I.ntp, defer, Ju, Fa, tsum, G, lane, rrow, teta, tw);
          }
        } else {
          vk_rows2<GM, TAN, (NW == 8 && GM <= 2) ? 3 : 2, SPLIT ? kKeep : kStream>(
              P.H + I.h_off, TAN ? P.Hd + I.h_off : nullptr, I.nt, I.ntp, U.qs, r0, r1, Xs, Us, red, Ju, Fa, tsum,
              G, lane, rrow, teta, tw);
        }
        if (NW > 1) {
#pragma unroll
          for (int g = 0; g < GM; ++g) {
            const int k4 = lane + kWave * g;
            if (g < G && k4 < nc) {
              st4(red + 4 * k4, Ju[g]);
              st4(red + I.ntp + 4 * k4, Fa[g]);
            }
          }
          if (lane == 0) red[2 * I.ntp] = tsum;
          __syncthreads();
          if (wave == 0) {
#pragma unroll
            for (int g = 0; g < GM; ++g) {
              const int k4 = lane + kWave * g;
              if (g < G && k4 < nc)
                for (int w = 1; w < NW; ++w) {
                  const float* o = L.red + w * P.red_floats;
                  Ju[g] = add4(Ju[g], ld4(o + 4 * k4));
                  Fa[g] = add4(Fa[g], ld4(o + I.ntp + 4 * k4));
                }
            }
            if (TAN)
              for (int w = 1; w < NW; ++w) tsum += L.red[w * P.red_floats + 2 * I.ntp];
          }
        }
        if (TAN && wave == 0 && lane == 0) {
          // theta partial of this unit: mode slot 0 of its theta accumulator
          acc_add(P.acc, 5, P.state_floats, U.state_off, {tsum, 0.f});
        }
      } else if (I.kind == KIND_TENSION && wave == 0) {
        // F = kappa lam x S, J u = kappa lam (u S + 2 x sum(lam x u))
        const float S = wave_sum(sx), T2 = 2.f * wave_sum(sxu);
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) {
            const float4 x4 = ld4(P.rec_x + ro + 4 * k4);
            const float4 l = ld4(P.lam + I.mode_off + 4 * k4);
            const float4 u4 = Ju[g];
            const float k = I.kappa;
            Fa[g] = make_float4(k * l.x * x4.x * S, k * l.y * x4.y * S, k * l.z * x4.z * S,
                                k * l.w * x4.w * S);
            Ju[g] = make_float4(k * l.x * fmaf(u4.x, S, x4.x * T2), k * l.y * fmaf(u4.y, S, x4.y * T2),
                                k * l.z * fmaf(u4.z, S, x4.z * T2), k * l.w * fmaf(u4.w, S, x4.w * T2));
          }
        }
      }
      if (wave == 0) {
        if (I.nslab == 1) {
          adj_post<GM>(P, I, U, n, Ju, Fa, G, lane);
        } else {
          // this instance's exchange region: [2][nslab][2 ntp] floats
          const v4i pr = buf_rsrc(P.part + 2 * I.part_off, 16 * I.nslab * I.ntp);
          const int dst = 8 * ((int)(rstep & 1) * I.nslab + U.slab) * I.ntp;
#pragma unroll
          for (int g = 0; g < GM; ++g) {
            const int k4 = lane + kWave * g;
            if (g < G && k4 < nc) {
              st4_coherent(pr, dst + 16 * k4, Ju[g]);
              st4_coherent(pr, dst + 4 * I.ntp + 16 * k4, Fa[g]);
            }
          }
          publish_fence();
          __builtin_amdgcn_wave_barrier();
          if (lane == 0)
            __hip_atomic_store(&P.ctr[I.ctr_off + U.slab], (unsigned int)(rstep + 1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __syncthreads();  // LDS reused by the next unit
    }
    for (int u = u0; u < u1; ++u) {
      const UnitDev U = P.unit[u];
      const InstDev I = P.inst[U.inst];
      if (I.nslab == 1) continue;
      if (wave == 0) {
        const bool ok = wait_slabs(P.ctr + I.ctr_off, I.nslab, (unsigned int)(rstep + 1), P.flags, P.timeout_ticks);
        if (lane == 0) L.flag[0] = ok ? 1 : 0;
      }
      __syncthreads();
      if (L.flag[0] == 0) return;  // every wave leaves together
      const int nc = I.ntp >> 2;
      const int G = (nc + kWave - 1) / kWave;
      const v4i pr = buf_rsrc(P.part + 2 * I.part_off, 16 * I.nslab * I.ntp);
      const int src = 8 * (int)(rstep & 1) * I.nslab * I.ntp;  // byte offset of this step's partials
      if (SPLIT && NW > 1 && I.nslab >= 2 * NW) {
        // many slabs: every wave sums every NW-th partial, wave 0 adds the
        // waves' sums
        consume_fence();
        float4 Ju[GM], F[GM];
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          Ju[g] = F[g] = f4(0.f);
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc) {
            Ju[g] = sum_slabs4_coherent(pr, src + 16 * k4, wave, NW, I.nslab, 8 * I.ntp);
            F[g] = sum_slabs4_coherent(pr, src + 4 * I.ntp + 16 * k4, wave, NW, I.nslab, 8 * I.ntp);
            st4(red + 4 * k4, Ju[g]);
            st4(red + I.ntp + 4 * k4, F[g]);
          }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
          for (int g = 0; g < GM; ++g) {
            const int k4 = lane + kWave * g;
            if (g < G && k4 < nc)
              for (int w = 1; w < NW; ++w) {
                const float* o = L.red + w * P.red_floats;
                Ju[g] = add4(Ju[g], ld4(o + 4 * k4));
                F[g] = add4(F[g], ld4(o + I.ntp + 4 * k4));
              }
          }
          adj_post<GM>(P, I, U, n, Ju, F, G, lane);
        }
      } else if (wave == 0) {
        consume_fence();
        float4 Ju[GM], F[GM];
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          Ju[g] = F[g] = f4(0.f);
          const int k4 = lane + kWave * g;
          if (g < G && k4 < nc)
            for (int t = 0; t < I.nslab; ++t) {
              Ju[g] = add4(Ju[g], ld4_coherent(pr, src + 8 * t * I.ntp + 16 * k4));
              F[g] = add4(F[g], ld4_coherent(pr, src + 8 * t * I.ntp + 4 * I.ntp + 16 * k4));
            }
        }
        adj_post<GM>(P, I, U, n, Ju, F, G, lane);
      }
      __syncthreads();  // flag reused
    }
  }
}

// Full tensor gradient of one segment: for in-plane row n (blockIdx.y) of job
// blockIdx.z, the 64 x 64 output tile blockIdx.x gets
//   out[n][i][j] -= sum_s a_i^s q_j^s,   a_i^s = (V_n . u)^s q_i^s + eta_n^s u_i^s,
// a product over the segment's steps: 16 steps of a and q staged in LDS per
// round, a 4 x 4 block of the tile per thread.
__global__ void __launch_bounds__(256) tensor_grad_kernel(const TGradJob* __restrict__ jobs,
                                                          const float* __restrict__ rec_x,
                                                          const float* __restrict__ urec,
                                                          const float* __restrict__ trec, int mode_floats,
                                                          int rows_total, int seg_len) {
  const TGradJob J = jobs[blockIdx.z];
  const int n = blockIdx.y;
  const int tiles = (J.nt + kTgTile - 1) / kTgTile;
  if (n >= J.nin || (int)blockIdx.x >= tiles * tiles) return;
  const int i0 = (blockIdx.x / tiles) * kTgTile, j0 = (blockIdx.x % tiles) * kTgTile;
  __shared__ float4 As4[kTgChunk][kTgTile / 4], Bs4[kTgChunk][kTgTile / 4];
  float* As = reinterpret_cast<float*>(As4);
  float* Bs = reinterpret_cast<float*>(Bs4);
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int c0 = 0; c0 < seg_len; c0 += kTgChunk) {
#pragma unroll
    for (int r = 0; r < (kTgChunk * kTgTile) / 256; ++r) {
      const int e = tid + 256 * r;
      const int sl = e / kTgTile, k = e % kTgTile;
      const int st = c0 + sl;
      float av = 0.f, bv = 0.f;
      if (st < seg_len) {
        const long long xo = (long long)st * mode_floats + J.mode_off;
        const long long to = (long long)st * 2 * rows_total + J.row_off + n;
        if (i0 + k < J.nt) av = trec[to + rows_total] * rec_x[xo + i0 + k] + trec[to] * urec[xo + i0 + k];
        if (j0 + k < J.nt) bv = rec_x[xo + j0 + k];
      }
      As[e] = av;
      Bs[e] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < kTgChunk; ++sl) {
      const float4 a = As4[sl][ty], b = Bs4[sl][tx];
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(av[x], bv[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int i = i0 + 4 * ty + x;
    if (i >= J.nt) continue;
    float* o = J.out + ((long long)n * J.nt + i) * J.nt;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int j = j0 + 4 * tx + y;
      if (j < J.nt) o[j] -= acc[x][y];
    }
  }
}

// Sets *bad when H[n][i][j] != H[n][j][i] for any entry (exact comparison);
// H is [nin][nt][nt].
__global__ void sym_check_kernel(const float* __restrict__ H, int nin, int nt, int* bad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)nt * nt;
  if (e >= per * nin) return;
  const long long n = e / per;
  const int i = (int)((e % per) / nt), j = (int)(e % nt);
  if (j <= i) return;
  if (H[n * per + (long long)i * nt + j] != H[n * per + (long long)j * nt + i]) atomicOr(bad, 1);
}

hipError_t launch_sym_check(const float* H, int nin, int nt, int* bad, hipStream_t s) {
  const long long total = (long long)nin * nt * nt;
  if (total < 1) return hipSuccess;
  hipLaunchKernelGGL(sym_check_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, H, nin, nt, bad);
  return hipGetLastError();
}

hipError_t launch_tensor_grad(const TGradJob* jobs, int n_jobs, int max_nin, int max_nt, const float* rec_x,
                              const float* urec, const float* trec, int mode_floats, int rows_total,
                              int seg_len, hipStream_t s) {
  if (n_jobs < 1 || max_nin < 1 || max_nt < 1 || seg_len < 1) return hipSuccess;
  const int tiles = (max_nt + kTgTile - 1) / kTgTile;
  hipLaunchKernelGGL(tensor_grad_kernel, dim3(tiles * tiles, max_nin, n_jobs), dim3(256), 0, s, jobs, rec_x,
                     urec, trec, mode_floats, rows_total, seg_len);
  return hipGetLastError();
}

// Adds the per-row records of one segment (steps in record order) to the
// float-float row accumulators acc[2][rows].
__global__ void row_sum_kernel(const float* rrec, int seg_len, int rows, float* acc) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  ff a{acc[r], acc[rows + r]};
  for (int s = 0; s < seg_len; ++s) a = ff_add(a, ff{rrec[(long long)s * rows + r], 0.f});
  acc[r] = a.hi;
  acc[rows + r] = a.lo;
}

// Copies checkpoint `slot` ([4][mode_floats]) into every unit's state and
// rewinds the step counter and the forward arrival words to `step`.
__global__ void restore_kernel(const float* ckpt, long long slot, int mode_floats, const InstDev* inst,
                               const UnitDev* unit, int n_units, float* state, int state_floats,
                               long long* step_base, long long step, unsigned int* ctr) {
  const int u = blockIdx.x;
  if (u >= n_units) return;
  const UnitDev U = unit[u];
  const InstDev I = inst[U.inst];
  if (threadIdx.x == 0) ctr[I.ctr_off + U.slab] = (unsigned int)step;
  const float* src = ckpt + slot * 4LL * mode_floats + I.mode_off;
  for (int k = threadIdx.x; k < I.ntp; k += blockDim.x)
    for (int a = 0; a < 4; ++a)
      state[(long long)a * state_floats + U.state_off + k] = src[(long long)a * mode_floats + k];
  if (u == 0 && threadIdx.x == 0) *step_base = step;
}

// gm: float4 column groups per lane (1, 2 or 4); nw: waves per workgroup (1 or 4).
// split: the launch's workgroups own one unit each and their waves share the
// unit's row blocks (latency-bound plans); only with four or eight waves.
hipError_t launch_grad(const GradParams& P, int gm, bool tangent, int nw, bool split, int n_wg, size_t lds,
                       hipStream_t s) {
#define GL(G, T, W, S) hipLaunchKernelGGL((grad_kernel<G, T, W, S>), dim3(n_wg), dim3(kWave * W), lds, s, P)
#define GL_NW(G, T)                                        \
  if (nw == 1) GL(G, T, 1, false);                         \
  else if (nw == 8) { if (split) GL(G, T, 8, true); else GL(G, T, 8, false); } \
  else { if (split) GL(G, T, 4, true); else GL(G, T, 4, false); }
#define GL_T(G) \
  if (tangent) { GL_NW(G, true) } else { GL_NW(G, false) }
  if (gm <= 1) {
    GL_T(1)
  } else if (gm <= 2) {
    GL_T(2)
  } else {
    GL_T(4)
  }
#undef GL_T
#undef GL_NW
#undef GL
  return hipGetLastError();
}

hipError_t grad_occupancy(int* blocks, int gm, bool tangent, int nw, bool split, size_t lds) {
#define GO(G, T, W, S) \
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, grad_kernel<G, T, W, S>, kWave * W, lds)
#define GO_NW(G, T)                                                         \
  {                                                                         \
    if (nw == 1) { GO(G, T, 1, false); }                                    \
    else if (nw == 8) { if (split) { GO(G, T, 8, true); } else { GO(G, T, 8, false); } } \
    else { if (split) { GO(G, T, 4, true); } else { GO(G, T, 4, false); } } \
  }
#define GO_T(G) \
  { if (tangent) { GO_NW(G, true) } else { GO_NW(G, false) } }
  if (gm <= 1) GO_T(1)
  if (gm <= 2) GO_T(2)
  GO_T(4)
#undef GO_T
#undef GO_NW
#undef GO
}

hipError_t launch_row_sum(const float* rrec, int seg_len, int rows, float* acc, hipStream_t s) {
  if (rows < 1) return hipSuccess;
  hipLaunchKernelGGL(row_sum_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, rrec, seg_len, rows, acc);
  return hipGetLastError();
}

hipError_t launch_restore(const float* ckpt, long long slot, int mode_floats, const InstDev* inst,
                          const UnitDev* unit, int n_units, float* state, int state_floats,
                          long long* step_base, long long step, unsigned int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(restore_kernel, dim3(n_units), dim3(256), 0, s, ckpt, slot, mode_floats, inst,
                     unit, n_units, state, state_floats, step_base, step, ctr);
  return hipGetLastError();
}

}  // namespace modal
