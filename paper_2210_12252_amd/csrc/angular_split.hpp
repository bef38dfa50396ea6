// Angular stage of H*X with the theta1 direction transformed instead of
// convolved, for grids where the m range covers most of a small theta1 grid
// (N1 = 32 or 48 points for 25 or 24 values of m).  The block of a radius
// is stored row by row (row stride ang_rs(N2), no column swizzle).
//
// The library runs it in FP32 arithmetic (FP32 and BF16 modes), where it
// measured faster than the convolution; the kernel itself is generic in T.
//
// Per radius and vector (Alg. 2, the product with V, Alg. 4): the mode block
// G_{m,n} (M rows of m) is transformed over theta2 row by row (the four-step
// P x P transform of k_angular_fast, slab elements moved straight between
// global memory and the registers of the row transforms), then each theta2
// column j is zero-padded from M to N1 values of m, transformed to the N1
// theta1 points, multiplied by the real V(theta1_i, theta2_j, r) / (N1 N2),
// transformed back and cropped to the M rows; the theta2 forward transform
// and the store to the slab close the vector.  Since the operator depends on
// m' - m only, the phase exp(i 2 pi m_min i / N1) of the first row cancels
// between the two column transforms, so block row m - m_min enters the
// column DFT at position m - m_min.  The result equals the convolution
// sum_m Vhat_j[m' - m] G[m] of k_angular_fast up to rounding, at
// O(N1 log N1) instead of M^2 operations per column.
//
// A column is transformed by C = 4 lanes of one wave (N1 = C Q): lane s
// holds rows s + C q, does the Q-point DFT over q, multiplies by
// exp(+2 pi i s k1 / N1), and after an exchange through the column's own LDS
// positions (wave-level ordering suffices) lane s holds k1 = s + C u for every
// s' and does C-point DFTs, which give theta1 points i = k1 + Q k2.  The
// forward transform mirrors these steps and leaves output row m1 + C m2 in
// lane m1, the layout the column was read in.  The block therefore has N1
// rows (the rows beyond M serve the exchanges), and one vector costs two
// block barriers.
#pragma once
#include "angular_fast.hpp"

namespace helic {

constexpr int SPLIT_C = 4;   // lanes per theta1 column

// Column transform of block column j, lane s (0 <= s < C) of its quad.
// The block is stored without the column swizzle of k_angular_fast (row
// stride ang_rs(N2)), so every access is one of two per-lane base addresses
// plus a compile-time row offset: c0 = column j at row s, c1 = column j at
// row s Q.  v[u * C + k2] = V at theta1 point (s + C u) + Q k2 of this
// column, already scaled by 1 / (N1 N2).  Rows >= MPAD read as zero and are
// not written.  All lanes of the wave call (act false: no LDS access).
template <typename T, int N1, int N2, int MPAD>
__device__ __forceinline__ void split_column(cplx<T>* A, const cplx<T>* tw1, int j, int s, bool act, const T* v) {
  constexpr int C = SPLIT_C, Q = N1 / C, U = Q / C;
  static_assert(C * Q == N1 && U * C == Q, "N1 must be a multiple of 16");
  constexpr int RS = ang_rs(N2);
  cplx<T>* c0 = A + s * RS + j;
  cplx<T>* c1 = A + s * Q * RS + j;
  cplx<T> x[Q];
  if (act) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (C * q >= MPAD) x[q] = cplx<T>{(T)0, (T)0};   // every lane's row is beyond M
      else if (C * q + C - 1 < MPAD) x[q] = c0[C * q * RS];
      else x[q] = s + C * q < MPAD ? c0[C * q * RS] : cplx<T>{(T)0, (T)0};
    }
    dft_reg<T, Q, true>(x);
#pragma unroll
    for (int k1 = 1; k1 < Q; ++k1) {
      cplx<T> w = tw1[s * k1];   // exp(-2 pi i s k1 / N1), s k1 < N1
      w.y = -w.y;
      x[k1] = cmul(x[k1], w);
    }
  }
  wave_sync();
  // exchange 1: Y[s][k1] at row s Q + k1 of the column
  if (act) {
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) c1[k1 * RS] = x[k1];
  }
  wave_sync();
  cplx<T> y[U][C];
  if (act) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s2 = 0; s2 < C; ++s2) y[u][s2] = c0[(s2 * Q + C * u) * RS];   // Y[s2][s + C u]
      dft_reg<T, C, true>(y[u]);   // theta1 points (s + C u) + Q k2
#pragma unroll
      for (int k2 = 0; k2 < C; ++k2) {
        const T f = v[u * C + k2];
        y[u][k2] = cplx<T>{y[u][k2].x * f, y[u][k2].y * f};
      }
      dft_reg<T, C, false>(y[u]);  // Z[k1 = s + C u][m1]
#pragma unroll
      for (int m1 = 1; m1 < C; ++m1) y[u][m1] = cmul(y[u][m1], tw1[(m1 * (s + C * u)) % N1]);
    }
  }
  wave_sync();
  // exchange 2: Z[k1][m1] at row m1 Q + k1
  if (act) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int m1 = 0; m1 < C; ++m1) c0[(m1 * Q + C * u) * RS] = y[u][m1];
    }
  }
  wave_sync();
  if (act) {
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) x[k1] = c1[k1 * RS];
    dft_reg<T, Q, false>(x);       // output rows s + C m2
  }
  wave_sync();
  if (act) {
#pragma unroll
    for (int m2 = 0; m2 < Q; ++m2) {
      if (C * m2 >= MPAD) continue;
      if (C * m2 + C - 1 < MPAD || s + C * m2 < MPAD) c0[C * m2 * RS] = x[m2];
    }
  }
}

// GH[v][r][mode] holds G on entry and H on exit (elements E: complex T, or
// bfloat16 pairs read and written in FP32 arithmetic).  Vs[r][i1][i2] is
// V / (N1 N2) (T).  blk_mode[(m - m_min) N2 + (n mod N2)] = mode index or -1.
// tw2g[t] = exp(-2 pi i t / N2), tw1g[t] = exp(-2 pi i t / N1).
// Work: blockIdx -> ipw consecutive (problem, radius, vector) items, as
// segments of one radius (V and the block -> mode table are loaded once per
// segment); the next vector's slab elements are loaded while the current one
// is transformed.  Registers are held to 4 waves per SIMD in FP32 (2 in
// FP64, where 3 would spill).
template <typename T, typename E, int N1, int N2, int MPAD, int NTF>
__global__ void __launch_bounds__(NTF, (sizeof(T) == 8 ? 2 : 4))
k_angular_split(E* __restrict__ GH, int nprob, int nvec, int n_r, const DProb* __restrict__ probs,
                const cplx<T>* __restrict__ tw2g, const cplx<T>* __restrict__ tw1g, int ipw) {
  constexpr int P = (N2 == 64) ? 8 : (N2 == 81) ? 9 : 0;
  static_assert(P > 0, "unsupported N2");
  static_assert(MPAD <= N1, "the m rows must fit the theta1 grid");
  constexpr int C = SPLIT_C, Q = N1 / C, U = Q / C;
  constexpr int RS = ang_rs(N2);
  constexpr int NCT = N2 * C;                          // column lanes
  constexpr int NPASS = (NCT + NTF - 1) / NTF;
  constexpr int RPW = 64 / P;
  static_assert(MPAD <= RPW * (NTF / 64), "one batch of rows");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);   // [N1][RS]
  cplx<T>* tw2 = A + N1 * RS;                          // [N2]
  cplx<T>* tw1 = tw2 + N2;                             // [N1]
  const int64_t per_prob = (int64_t)n_r * nvec;
  const int64_t total = per_prob * nprob;
  const int nwg = (int)((total + ipw - 1) / ipw);
  const int slot = xcd_slot(nwg);
  if (slot >= nwg) return;
  int64_t it = (int64_t)slot * ipw;
  const int64_t it_end = total < it + ipw ? total : it + ipw;
  const int t = threadIdx.x;
  for (int i = t; i < N2; i += NTF) tw2[i] = tw2g[i];
  for (int i = t; i < N1; i += NTF) tw1[i] = tw1g[i];
  __syncthreads();
  const int wv = t >> 6;
  // row-transform lane: row rrow, position rp
  const int rrow = wv * RPW + (t & 63) / P, rp = (t & 63) % P;
  const bool ract = (t & 63) < RPW * P && rrow < MPAD;
  while (it < it_end) {
    const int pi = (int)(it / per_prob);
    const int rem = (int)(it - pi * per_prob);
    const int r = rem / nvec, v0 = rem - r * nvec;
    const int v1 = (int)(nvec < v0 + (it_end - it) ? nvec : v0 + (it_end - it));
    it += v1 - v0;
    const DProb& pb = probs[pi];
    const T* vs = reinterpret_cast<const T*>(pb.Vs) + (int64_t)r * N1 * N2;
    T vr[NPASS][Q];
#pragma unroll
    for (int ps = 0; ps < NPASS; ++ps) {
      const int ct = ps * NTF + t, j = ct / C, s = ct % C;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k2 = 0; k2 < C; ++k2)
          vr[ps][u * C + k2] = ct < NCT ? vs[(s + C * u + Q * k2) * N2 + j] : (T)0;
    }
    int idx[P];
#pragma unroll
    for (int q = 0; q < P; ++q) idx[q] = ract ? pb.blk_mode[rrow * N2 + rp + P * q] : -1;
    cplx<T> xin[P];
    auto fetch = [&](int v) {
      const E* slab = GH + slab_off(pb, nvec, n_r, v, r);
#pragma unroll
      for (int q = 0; q < P; ++q) xin[q] = idx[q] >= 0 ? eload<T>(slab + idx[q]) : cplx<T>{(T)0, (T)0};
    };
    fetch(v0);
    for (int v = v0; v < v1; ++v) {
      row_idft_from_regs<T, N2, P, NTF, MPAD, 0, true, false>(A, tw2, xin);
      if (v + 1 < v1) fetch(v + 1);
      __syncthreads();
#pragma unroll
      for (int ps = 0; ps < NPASS; ++ps) {
        if (ps * NTF + wv * 64 < NCT) {                // wave-uniform
          const int ct = ps * NTF + t;
          split_column<T, N1, N2, MPAD>(A, tw1, ct / C, ct % C, ct < NCT, vr[ps]);
        }
      }
      __syncthreads();
      cplx<T> xout[P];
      row_dft_to_regs<T, N2, P, NTF, MPAD, 0, true, false>(A, tw2, xout);
      E* slab = GH + slab_off(pb, nvec, n_r, v, r);
      if (ract) {
#pragma unroll
        for (int q = 0; q < P; ++q)
          if (idx[q] >= 0) estore(slab + idx[q], xout[q]);
      }
    }
  }
}

}  // namespace helic
