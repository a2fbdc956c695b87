// Adjoint of the FP32 matrix-core evaluation: d ln L_t / d theta for the
// seven parameters (alpha, delta, psi, iota, phi, D, tau).
//
// With p_j the softmax weights of the window log-likelihoods (p_j = exp(ell_j)
// / sum exp(ell)), d ln L_t = sum_j p_j d ell_j, and d ell_j splits into
//   * the coefficients a_k: Re(conj(da_k) (G_k - U_k a_k / 2)) - Re(da_k V_k a_k) / 2
//     with G_k = sum_j p_j Qtilde_k(j) = sum_r c_k[r] Q_k[r] and
//     c_k[r] = sum_q w_q(mu_k) p_{r - P - 1 - n_k - q}   (the interpolation's transpose);
//   * the arrival time of detector k: f_s H_k d(dt_k) with
//     H_k = sum_j p_j Re(a_k^dag Qtilde'_k(j)), Qtilde' using the derivative weights;
// (App. D Eq. (def:lnL:Decomposed) differentiated; no separate passage of the
// paper covers the gradient).
//
// mfma_bwd_kernel takes the work units of the forward evaluation and makes
// one sweep over the rows: it recomputes z_k (the MFMA contraction), forms
// the softmax weights p_j online (unnormalized, against a running reference,
// as in a streaming softmax), accumulates H_k from the derivative
// interpolation, spreads p onto rows as c_k (through a small LDS ring of p
// per sample) and accumulates G_k = Q_k^T c_k as a second MFMA contraction
// whose A operand is the staged block of Q read transposed; the sums are
// normalized at the end, which also gives ln L_t.
// chain_kernel then applies the chain rule in FP64, one thread per sample.
#include "common.h"
#include "internal.h"
#include "mfma_tile.h"

#include <algorithm>

namespace rift {

constexpr int kRZ = 52;  // z ring row: two 16-row slots, slot 0 again at 32 (48 rows), padded for banks
constexpr int kRP = 52;  // p ring of a sample: the same arrangement over window blocks

template <int T, int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) mfma_bwd_kernel(MfmaArgs a, int item_lo, int item_hi, int cls) {
  constexpr int E = 4 * T, J = T / 4, R = T % 4;
  constexpr int JA = J > 0 ? J : 1, RA = R > 0 ? R : 1;
  constexpr int ES = stage_stride<T>();
  constexpr int SF = K * kTS * ES + 16;  // one staged block (+16: reads of the last row's padding)
  constexpr int MT = (E + 15) / 16;      // 16-element tiles of G
  __shared__ __align__(16) float ring_all[kWaves * K * kTS * kRZ];
  __shared__ __align__(16) float pring_all[kWaves * kTS * kRP];
  __shared__ __align__(16) float stage[3 * SF];  // block b in buffer b % 3
  __shared__ WorkUnit unit_sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float *ring = ring_all + wave * (K * kTS * kRZ);  // [det][sample][kRZ]
  float *pring = pring_all + wave * (kTS * kRP);     // [sample][kRP]
  const int s = lane & 15, g = lane >> 4;
  const uint32_t u_lo = a.item_units[item_lo], u_hi = a.item_units[item_hi];
  const int tid = threadIdx.x;
  const bool st_on = tid < 16 * T;
  const uint32_t st_goff = 16u * (uint32_t)tid;
  const int st_loff = (tid / T) * ES + 4 * (tid % T);

  for (;;) {
    if (tid == 0) {
      const uint32_t u = u_lo + atomicAdd(&a.ctl[1 + cls], 1u);
      WorkUnit w;
      if (u < u_hi) {
        w = a.unit[u];
      } else {
        w.tile = 0xffffffffu;
        w.ntiles = 0;
        w.key = 0;
      }
      unit_sh = w;
    }
    __syncthreads();
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(unit_sh.tile);
    const int ntiles = __builtin_amdgcn_readfirstlane(unit_sh.ntiles);
    uint32_t key = __builtin_amdgcn_readfirstlane(unit_sh.key);
    if (t0 == 0xffffffffu) break;
    const bool active = wave < ntiles;
    const uint32_t t = t0 + (active ? wave : 0);
    const int it = __builtin_amdgcn_readfirstlane(a.tile_item[t0]);
    const PointDev &p = a.pts[a.items.point[it]];
    const int NT = p.n_t, P = p.pad, Lpad = p.Lpad;
    const RIFT_GLOBAL float *qk[K];
    int lo_k[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int q = (int)(key % (uint32_t)p.nq);
      key /= (uint32_t)p.nq;
      lo_k[k] = q * p.bin_w - P;
      qk[k] = gp(uniform_ptr(p.Qm + (size_t)(k * Lpad + P + lo_k[k]) * E));
    }
    const int64_t top = a.item_cop[it] + (int64_t)(t - a.item_tiles[it]) * K * E * kTS;
    const RIFT_GLOBAL CoefTile *ct = gp(a.ctile + t);
    const int flag = active ? ct->flag[s] : 0;
    const int col = ct->col[s];
    const float Bf = active ? ct->B[s] : 0.f;
    float Bop[K][T];
    b_operands<T, K>(gp(a.cop + top + s), ct, s, g, active, Bop);
    float w[K][4], wd[K][4];
    int sh[K];
    bool valid = flag == 1;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const float mu = ct->mu[k][s];
      cr_weights<float>(mu, w[k]);
      cr_dweights<float>(mu, wd[k]);
      sh[k] = valid ? ct->n[k][s] - lo_k[k] : 0;
      if (sh[k] < 0 || sh[k] > kTS - 3) {
        valid = false;
        sh[k] = 0;
      }
    }
    const int JB = (NT + 15) >> 4;
    const int rem = NT - 16 * (JB - 1);
    float last_pen[4];
#pragma unroll
    for (int i = 0; i < 4; i++) last_pen[i] = (4 * g + i < rem) ? 0.f : -INFINITY;

    f4 pre[K];
    auto stage_load = [&](int blk) {
      if (st_on) {
        const uint32_t ob = (uint32_t)(64 * E) * (uint32_t)blk + st_goff;
#pragma unroll
        for (int k = 0; k < K; k++) pre[k] = *(const RIFT_GLOBAL f4 *)((const RIFT_GLOBAL char *)qk[k] + ob);
      }
    };
    auto stage_store = [&](int buf) {
      if (st_on) {
#pragma unroll
        for (int k = 0; k < K; k++) *(f4 *)(&stage[buf * SF + k * kTS * ES + st_loff]) = pre[k];
      }
    };
    // block b on the matrix cores -> z ring slot b % 2 (slot 0 also at 32)
    auto product = [&](int b) {
      const float *sb = &stage[(b % 3) * SF + s * ES];
      f4 Aq[K][JA];
      float At[K][RA];
#pragma unroll
      for (int k = 0; k < K; k++) {
#pragma unroll
        for (int j = 0; j < J; j++) Aq[k][j] = *(const f4 *)(sb + k * kTS * ES + 16 * j + 4 * g);
#pragma unroll
        for (int r = 0; r < R; r++) At[k][r] = sb[k * kTS * ES + 16 * J + 4 * r + g];
      }
      f4 acc[K];
#pragma unroll
      for (int tt = 0; tt < T; tt++)
#pragma unroll
        for (int k = 0; k < K; k++) {
          const float av = tt < 4 * J ? Aq[k][tt < 4 * J ? tt >> 2 : 0][tt & 3] : At[k][tt < 4 * J ? 0 : tt - 4 * J];
          acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Bop[k][tt], tt == 0 ? f4{0.f, 0.f, 0.f, 0.f} : acc[k], 0,
                                                        0, 0);
        }
      float *wp = ring + s * kRZ + 4 * g + 16 * (b & 1);
#pragma unroll
      for (int k = 0; k < K; k++) {
        *(f4 *)(wp + k * kTS * kRZ) = acc[k];
        if ((b & 1) == 0) *(f4 *)(wp + k * kTS * kRZ + 32) = acc[k];
      }
    };
    // window samples 16 c + 4 g + i of block c: ell + B - m_ref (base 2) and,
    // when wanted, the derivative interpolation zd_k.  The quadratic term B is
    // the same for every window sample: it stays out of the softmax (whose
    // weights it does not change) and enters ln L_t once at the end, so the
    // window values carry the rounding of the data term only.
    float m_ref = 0.f;
    auto interp = [&](int c, float (&ell)[4], float (&zd)[K][4], bool want_d) {
      const float base = -m_ref;
#pragma unroll
      for (int i = 0; i < 4; i++) ell[i] = (c == JB - 1) ? base + last_pen[i] : base;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const float *zr = ring + (k * kTS + s) * kRZ + 16 * (c & 1) + 4 * g + sh[k];
        float z[7];
#pragma unroll
        for (int o = 0; o < 7; o++) z[o] = zr[o];
#pragma unroll
        for (int i = 0; i < 4; i++) {
          ell[i] = fmaf(w[k][0], z[i], ell[i]);
          ell[i] = fmaf(w[k][1], z[i + 1], ell[i]);
          ell[i] = fmaf(w[k][2], z[i + 2], ell[i]);
          ell[i] = fmaf(w[k][3], z[i + 3], ell[i]);
          if (want_d)
            zd[k][i] = wd[k][0] * z[i] + wd[k][1] * z[i + 1] + wd[k][2] * z[i + 2] + wd[k][3] * z[i + 3];
        }
      }
    };

    // ---- one sweep: z_k, then per window block ell_j, the unnormalized
    // softmax weights p_j = 2^(ell_j + B - m_ref), H_k, c_k and G_k = Q_k^T c_k.
    // m_ref is shared by the 4 lanes of a sample (the G products and the
    // rows' taps mix their p): the first window block's maximum of ell + B, moved only
    // when a block's maximum exceeds it by 64, and then every sum kept so far
    // (G, H, the sum of p and the p of the previous block in the ring) is
    // scaled by 2^(m_ref - m_new).  At the end all of them are divided by the
    // sum of p, which also gives ln L_t.
    float s_run = 0.f;
    // Where the window's mass lies (for the FP64 refinement): the three
    // largest block maxima (t1 >= t2 >= t3, blocks i1, i2, i3) and the
    // largest maximum of every other block (rest)
    constexpr float kRefD2 = kRefineNats * 1.4426950408889634f;  // base 2
    float t1 = -INFINITY, t2 = -INFINITY, t3 = -INFINITY, rest = -INFINITY;
    int i1 = 0, i2 = 0, i3 = 0;
    float hsum[K];
#pragma unroll
    for (int k = 0; k < K; k++) hsum[k] = 0.f;
    f4 gacc[K][MT];
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
      for (int mt = 0; mt < MT; mt++) gacc[k][mt] = f4{0.f, 0.f, 0.f, 0.f};
    float *pr = pring + s * kRP;  // this lane's sample
    // p of window block -1 (slot 1) is zero
    *(f4 *)(pr + 16 + 4 * g) = f4{0.f, 0.f, 0.f, 0.f};
    // G += Q_k^T c_k over row block rb (stage buffer rb % 3); p of window
    // blocks rb - 1 and rb are in the p ring
    auto gproduct = [&](int rb) {
      const float *sg = &stage[(rb % 3) * SF + 4 * g * ES + s];  // row 4 g (+ ks), element s (+ 16 mt)
#pragma unroll
      for (int k = 0; k < K; k++) {
        // c_k at rows 16 rb + 4 g + ks (ks < 4): taps on p_j, j = row - sh - o
        const float *pp = pr + 16 * ((rb + 1) & 1) + 13 + 4 * g - sh[k];  // p of j = 16 rb + 4 g - sh - 3
        float pv[7];
#pragma unroll
        for (int o = 0; o < 7; o++) pv[o] = pp[o];
        float c[4];
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
          c[ks] = w[k][0] * pv[ks + 3] + w[k][1] * pv[ks + 2] + w[k][2] * pv[ks + 1] + w[k][3] * pv[ks];
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
#pragma unroll
          for (int mt = 0; mt < MT; mt++) {
            const float av = sg[k * kTS * ES + ks * ES + 16 * mt];
            gacc[k][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, c[ks], gacc[k][mt], 0, 0, 0);
          }
      }
    };
    stage_load(0);
    stage_store(0);
    __syncthreads();
    for (int b = 0; b <= JB; b++) {
      stage_load(min(b + 1, JB));
      if (active) {
        product(b);
        wave_sync();
        if (b >= 1) {
          const int c = b - 1;
          float ell[4], zd[K][4];
          interp(c, ell, zd, true);
          float cmax = fmaxf(fmaxf(ell[0], ell[1]), fmaxf(ell[2], ell[3]));
          cmax = fmaxf(cmax, __shfl_xor(cmax, 16));
          cmax = fmaxf(cmax, __shfl_xor(cmax, 32));
          {
            const float v = cmax > -3.0e38f ? cmax + m_ref : -INFINITY;
            if (v > t3) {
              rest = fmaxf(rest, t3);
              if (v > t1) {
                t3 = t2; i3 = i2;
                t2 = t1; i2 = i1;
                t1 = v; i1 = c;
              } else if (v > t2) {
                t3 = t2; i3 = i2;
                t2 = v; i2 = c;
              } else {
                t3 = v; i3 = c;
              }
            } else {
              rest = fmaxf(rest, v);
            }
          }
          if ((c == 0 || cmax > 64.f) && cmax > -3.0e38f) {  // uniform over a sample's lanes
            if (c > 0) {
              const float f = __builtin_amdgcn_exp2f(-cmax);
              s_run *= f;
#pragma unroll
              for (int k = 0; k < K; k++) {
                hsum[k] *= f;
#pragma unroll
                for (int mt = 0; mt < MT; mt++) gacc[k][mt] *= f;
              }
              float *pq = pr + 16 * ((c - 1) & 1) + 4 * g;  // this lane's p of block c - 1
              f4 pv = *(f4 *)pq * f;
              *(f4 *)pq = pv;
              if (((c - 1) & 1) == 0) *(f4 *)(pq + 32) = pv;
            }
            m_ref += cmax;
#pragma unroll
            for (int i = 0; i < 4; i++) ell[i] -= cmax;
          }
          float pj[4];
#pragma unroll
          for (int i = 0; i < 4; i++) pj[i] = __builtin_amdgcn_exp2f(ell[i]);
#pragma unroll
          for (int i = 0; i < 4; i++) s_run += pj[i];
#pragma unroll
          for (int k = 0; k < K; k++)
#pragma unroll
            for (int i = 0; i < 4; i++) hsum[k] = fmaf(pj[i], zd[k][i], hsum[k]);
          float *pw = pr + 16 * (c & 1) + 4 * g;
          *(f4 *)pw = f4{pj[0], pj[1], pj[2], pj[3]};
          if ((c & 1) == 0) *(f4 *)(pw + 32) = f4{pj[0], pj[1], pj[2], pj[3]};
          wave_sync();
          gproduct(c);
        }
      }
      stage_store((b + 1) % 3);
      __syncthreads();
    }
    // the softmax normalizer (base 2) of the sample, from its 4 lanes
    float ssum = s_run;
    ssum += __shfl_xor(ssum, 16);
    ssum += __shfl_xor(ssum, 32);
    const float L2 = (m_ref - Bf) + __log2f(ssum);
    float lt = L2 * kLn2f - __logf((float)NT);
    if (!valid || !isfinite(lt)) {
      lt = NAN;
      valid = false;
    }
    const float inv = 1.f / ssum;

    if (active) {
      // the last row block: window block JB does not exist (p = 0)
      float *pw = pr + 16 * (JB & 1) + 4 * g;
      *(f4 *)pw = f4{0.f, 0.f, 0.f, 0.f};
      if ((JB & 1) == 0) *(f4 *)(pw + 32) = f4{0.f, 0.f, 0.f, 0.f};
      wave_sync();
      gproduct(JB);
      // H_k: the 4 lanes of a sample; z is in base-2 units (times log2 e)
      if (flag != 0) {
        RIFT_GLOBAL float *ho = gpw(a.hop + (size_t)t * (kMaxDet * kTS));
#pragma unroll
        for (int k = 0; k < K; k++) {
          float h = hsum[k];
          h += __shfl_xor(h, 16);
          h += __shfl_xor(h, 32);
          if (g == 0) ho[k * kTS + s] = valid ? h * inv * kLn2f : NAN;
        }
        // G_k[e = 16 mt + 4 g + v] of sample s
        RIFT_GLOBAL float *go = gpw(a.gop + top);
#pragma unroll
        for (int k = 0; k < K; k++)
#pragma unroll
          for (int mt = 0; mt < MT; mt++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
              const int e = 16 * mt + 4 * g + v;
              if (e < E) go[((size_t)k * E + e) * kTS + s] = gacc[k][mt][v] * inv;
            }
        if (g == 0) {
          if (a.jrng) {
            // the blocks within kRefD2 of the sample's maximum, when every
            // other block lies further below it: (blocks, count) or count 0
            const float thr = t1 - kRefD2;
            const int nb = (t2 >= thr ? (t3 >= thr ? 3 : 2) : 1);
            const bool ok = valid && t1 > -3.0e38f && rest < thr && i1 < 65536 && i2 < 65536 && i3 < 65536;
            if (ok) {
              const uint32_t r = atomicAdd(&a.ctl[kCtlRefine], 1u);
              RIFT_GLOBAL int *jo = gpw(a.jrng) + 4 * (size_t)r;
              jo[0] = (int)(t * kTS + s);
              jo[1] = i1 | ((nb > 1 ? i2 : 0) << 16);
              jo[2] = (nb > 2 ? i3 : 0) | (nb << 16);
            }
          }
          if (a.lnL) gpw(a.lnL)[col] = lt;
          if (a.lnw) gpw(a.lnw)[col] = lt + (a.ln_ratio ? gp(a.ln_ratio)[col] : 0.f);
        }
      }
    }
  }
}

// ---- chain rule, FP64, one thread per sorted slot --------------------------
// Point constants come through the constant address space (a block is 4 whole
// tiles of one point).  Harmonics and their iota derivatives from the
// polynomial tables: Y = s^par P(u) e^{i m phi} with s = sin(iota)/2 and
// u = cos^2(iota/2), so dY/diota = (par cos(iota)/2 P(u) - s^(par+1) P'(u))
// e^{i m phi}, with P and P' by one Horner pass.
template <int MC>
__global__ void __launch_bounds__(64) chain_kernel(MfmaArgs a, int item_lo, int item_hi) {
  constexpr int YR = MC > 0 ? MC : kMaxModes;
  const int64_t t_lo = a.item_tiles[item_lo], t_hi = a.item_tiles[item_hi];
  const int64_t t_blk = t_lo + 4 * (int64_t)blockIdx.x;
  if (t_blk >= t_hi) return;  // whole block (items hold whole blocks of 4 tiles)
  const int64_t pos = t_blk * kTS + threadIdx.x;
  const int64_t t = pos / kTS;
  const int s = (int)(pos % kTS);
  const SampleRec rec = a.rec[pos];
  if (rec.flag == 0) return;  // padding
  const int it = __builtin_amdgcn_readfirstlane(a.tile_item[t_blk]);
  const int pt = __builtin_amdgcn_readfirstlane(a.items.point[it]);
  const RIFT_CONST PointDev &p = *cp(a.pts + pt);
  const int K = p.K, E = 2 * p.Mp;
  const int M = MC > 0 ? MC : p.M;
  const int64_t col = rec.col;
  const RIFT_GLOBAL float *gk = gp(a.gop + a.item_cop[it] + (int64_t)(t - a.item_tiles[it]) * K * E * kTS + s);
  const RIFT_GLOBAL float *hk = gp(a.hop + (size_t)t * (kMaxDet * kTS) + s);
  double out[7] = {0, 0, 0, 0, 0, 0, 0};
  bool ok = rec.flag == 1;
  for (int k = 0; k < K && ok; k++) ok = isfinite(hk[k * kTS]);
  if (ok) {
    double th[7];
#pragma unroll
    for (int d = 0; d < 7; d++) th[d] = (double)rec.th[d];
    const double x = p.d_ref / th[RIFT_DIST];
    SkyTrig tr = sky_trig(th[RIFT_ALPHA], th[RIFT_DELTA], th[RIFT_PSI], p.gmst);
    double ci, si, c1, s1;
    sincos(0.5 * th[RIFT_IOTA], &si, &ci);
    sincos(th[RIFT_PHI], &s1, &c1);
    const double u = ci * ci, hs = si * ci, hc = 0.5 * (ci * ci - si * si);
    // Y_m (and, with dy, dY_m / d iota) of mode m
    auto mode = [&](int m, double &yr, double &yi, double *dyr, double *dyi) {
      const int deg = p.hdeg[m];
      double P = p.hpoly[m][deg], dP = 0.0;
      for (int j = deg - 1; j >= 0; j--) {
        dP = fma(dP, u, P);
        P = fma(P, u, p.hpoly[m][j]);
      }
      double y, dy;
      if (p.hpar[m]) {
        y = hs * P;
        dy = hc * P - hs * hs * dP;
      } else {
        y = P;
        dy = -hs * dP;
      }
      const int em = p.em[m], am = em < 0 ? -em : em;
      double cr = 1.0, cim = 0.0;
      for (int q = 0; q < am; q++) {
        double nr = cr * c1 - cim * s1;
        cim = cr * s1 + cim * c1;
        cr = nr;
      }
      if (em < 0) cim = -cim;
      yr = y * cr;
      yi = y * cim;
      if (dyr) {
        *dyr = dy * cr;
        *dyi = dy * cim;
      }
    };
    // Y_m in registers (the U Y and V Y products use all of them); Y_m and
    // dY_m / d iota again, one mode at a time, in the loop below
    double Yr[YR], Yi[YR];
#pragma unroll
    for (int m = 0; m < YR; m++) {
      Yr[m] = Yi[m] = 0.0;
      if (m < M) mode(m, Yr[m], Yi[m], nullptr, nullptr);
    }
    const double dn_a[3] = {-tr.cd * tr.sh, tr.cd * tr.ch, 0.0};
    const double dn_d[3] = {-tr.sd * tr.ch, -tr.sd * tr.sh, tr.cd};
    const RIFT_CONST double *Uc = cp(p.U);
    const RIFT_CONST double *Vc = p.V ? cp(p.V) : nullptr;
#pragma unroll 1
    for (int k = 0; k < K; k++) {
      double D[9], rc[3];
#pragma unroll
      for (int i = 0; i < 9; i++) D[i] = p.D[k][i];
#pragma unroll
      for (int i = 0; i < 3; i++) rc[i] = p.rc[k][i];
      double Fp, Fc, dFa[2], dFd[2];
      antenna(D, tr, Fp, Fc, dFa, dFd);
      const double H = (double)hk[k * kTS];
      const double ddt_a = -(rc[0] * dn_a[0] + rc[1] * dn_a[1] + rc[2] * dn_a[2]);
      const double ddt_d = -(rc[0] * dn_d[0] + rc[1] * dn_d[1] + rc[2] * dn_d[2]);
      out[RIFT_ALPHA] += H * p.f_s * ddt_a;
      out[RIFT_DELTA] += H * p.f_s * ddt_d;
      out[RIFT_TAU] += H * p.f_s;
#pragma unroll 1
      for (int m = 0; m < M; m++) {
        double yr, yi, dyr, dyi;
        mode(m, yr, yi, &dyr, &dyi);
        const int em = p.em[m];
        // (U a)_m = x F_k (U Y)_m, (V a)_m = x F_k (V Y)_m
        const RIFT_CONST double *U = Uc + ((size_t)k * M + m) * M * 2;
        double uyr = 0.0, uyi = 0.0, vyr = 0.0, vyi = 0.0;
#pragma unroll
        for (int mp = 0; mp < YR; mp++) {
          if (mp >= M) break;
          const double ur = U[2 * mp], ui = U[2 * mp + 1];
          uyr = fma(-ui, Yi[mp], fma(ur, Yr[mp], uyr));
          uyi = fma(ui, Yr[mp], fma(ur, Yi[mp], uyi));
        }
        if (Vc) {
          const RIFT_CONST double *V = Vc + ((size_t)k * M + m) * M * 2;
#pragma unroll
          for (int mp = 0; mp < YR; mp++) {
            if (mp >= M) break;
            const double vr = V[2 * mp], vi = V[2 * mp + 1];
            vyr = fma(-vi, Yi[mp], fma(vr, Yr[mp], vyr));
            vyi = fma(vi, Yr[mp], fma(vr, Yi[mp], vyi));
          }
        }
        const double uar = x * (Fp * uyr - Fc * uyi), uai = x * (Fp * uyi + Fc * uyr);
        const double var = x * (Fp * vyr - Fc * vyi), vai = x * (Fp * vyi + Fc * vyr);
        const double Gr = (double)gk[((size_t)k * E + 2 * m) * kTS], Gi = (double)gk[((size_t)k * E + 2 * m + 1) * kTS];
        const double er = Gr - 0.5 * uar, ei = Gi - 0.5 * uai;
        auto contrib = [&](double dar, double dai) { return dar * er + dai * ei - 0.5 * (dar * var - dai * vai); };
        out[RIFT_ALPHA] += contrib(x * (dFa[0] * yr - dFa[1] * yi), x * (dFa[0] * yi + dFa[1] * yr));
        out[RIFT_DELTA] += contrib(x * (dFd[0] * yr - dFd[1] * yi), x * (dFd[0] * yi + dFd[1] * yr));
        const double Fpr = 2.0 * Fc, Fpi = -2.0 * Fp;  // dF / dpsi = -2 i F
        out[RIFT_PSI] += contrib(x * (Fpr * yr - Fpi * yi), x * (Fpr * yi + Fpi * yr));
        out[RIFT_IOTA] += contrib(x * (Fp * dyr - Fc * dyi), x * (Fp * dyi + Fc * dyr));
        const double iyr = -em * yi, iyi = em * yr;
        out[RIFT_PHI] += contrib(x * (Fp * iyr - Fc * iyi), x * (Fp * iyi + Fc * iyr));
        const double ar = x * (Fp * yr - Fc * yi), ai = x * (Fp * yi + Fc * yr);
        out[RIFT_DIST] += contrib(-ar / th[RIFT_DIST], -ai / th[RIFT_DIST]);
      }
    }
  }
  const double gi = a.gin ? (double)gp(a.gin)[col] : 1.0;
#pragma unroll
  for (int d = 0; d < 7; d++) gpw(a.grad)[d * a.stride + col] = ok ? (float)(gi * out[d]) : NAN;
}

template <int T, int K>
static void launch_bwd_tk(const MfmaArgs &a, int lo, int hi, int cls, hipStream_t st) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mfma_bwd_kernel<T, K>, 256, 0) != hipSuccess || nb < 1)
      nb = 1;
    per_cu = nb;
  }
  const int grid = std::max(1, a.grid / 4 * per_cu);
  hipLaunchKernelGGL((mfma_bwd_kernel<T, K>), dim3(grid), dim3(256), 0, st, a, lo, hi, cls);
}

template <int T>
static void launch_bwd_class(const MfmaArgs &a, int K, int lo, int hi, int cls, hipStream_t st) {
  if (K == 1) launch_bwd_tk<T, 1>(a, lo, hi, cls, st);
  else if (K == 2) launch_bwd_tk<T, 2>(a, lo, hi, cls, st);
  else launch_bwd_tk<T, 3>(a, lo, hi, cls, st);
}

hipError_t mfma_backward(const MfmaArgs &a, const int *class_T, const int *class_K, const int *class_item0,
                         int n_classes, const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles,
                         int n_mclasses, hipStream_t st, const Fanout &fo, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.total <= 0) return hipSuccess;
  hipError_t e = mfma_prepare(a, mclass_M, mclass_item0, mclass_tiles, n_mclasses, st);
  if (e != hipSuccess) return e;
  if (ev0) (void)hipEventRecord(ev0, st);
  fan_fork(fo, st, n_classes);
  for (int c = 0; c < n_classes; c++) {
    hipStream_t sc = fan_stream(fo, st, c);
    const int lo = class_item0[c], hi = class_item0[c + 1];
    const int K = class_K[c];
    switch (class_T[c]) {
#define RIFT_T_CASE(TT) \
  case TT: launch_bwd_class<TT>(a, K, lo, hi, c, sc); break;
      RIFT_T_CASE(1) RIFT_T_CASE(2) RIFT_T_CASE(3) RIFT_T_CASE(4) RIFT_T_CASE(5) RIFT_T_CASE(6) RIFT_T_CASE(7)
      RIFT_T_CASE(8) RIFT_T_CASE(9) RIFT_T_CASE(10) RIFT_T_CASE(11) RIFT_T_CASE(12) RIFT_T_CASE(13)
      RIFT_T_CASE(14) RIFT_T_CASE(15) RIFT_T_CASE(16)
#undef RIFT_T_CASE
      default: return hipErrorInvalidValue;
    }
  }
  fan_join(fo, st, n_classes);
  if (ev1) (void)hipEventRecord(ev1, st);
  for (int c = 0; c < n_mclasses; c++) {
    const int lo = mclass_item0[c], hi = mclass_item0[c + 1];
    const dim3 grid((unsigned)(((int64_t)kTS * mclass_tiles[c] + 63) / 64));
    switch (mclass_M[c] < 0 ? -mclass_M[c] : mclass_M[c]) {
      case 2: hipLaunchKernelGGL(chain_kernel<2>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 5: hipLaunchKernelGGL(chain_kernel<5>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 9: hipLaunchKernelGGL(chain_kernel<9>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 21: hipLaunchKernelGGL(chain_kernel<21>, grid, dim3(64), 0, st, a, lo, hi); break;
      default: hipLaunchKernelGGL(chain_kernel<0>, grid, dim3(64), 0, st, a, lo, hi); break;
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return refine_backward(a, st);
}

}  // namespace rift
