// Angular stage of H*X for grids whose theta1 size N1 is small: the 2D DFTs
// run as row transforms over theta2 (N2 = PA * PB, four-step with the PB- and
// PA-point DFTs in registers and one exchange through LDS) and column
// transforms over theta1 (the whole N1-point column in one thread's
// registers), with the real potential applied on the grid between the two
// column transforms (Alg. 2, the product with V, Alg. 4).  Used where the
// m range fills most of the theta1 grid, so the theta1 FFT is cheaper than the
// Toeplitz convolution of k_angular_fast.
#pragma once
#include "angular_fast.hpp"

namespace helic {

// Row stride (complex elements) of the grid block.
__host__ __device__ constexpr int grid_rs(int n2) { return n2 + 1; }

// In-place length N2 = PA * PB DFT of rows 0..rows-1 of A (row stride RS),
// TPR = max(PA, PB) threads per row, rows packed whole into waves (64 / TPR
// rows per wave) so the exchange needs only wave-level ordering.  x[p + PA q]
// -> PB-point DFT over q per thread p -> twiddle exp(s 2 pi i p k1 / N2) ->
// exchange -> PA-point DFT over p per thread k1 -> X[k1 + PB k2].  A must be
// synchronised on entry; it is on exit.
template <typename T, int N2, int PA, int PB, int NTF, bool INV>
__device__ __forceinline__ void row_dft2(cplx<T>* A, int rows, const cplx<T>* tw) {
  static_assert(PA * PB == N2, "row transform expects N2 = PA * PB");
  constexpr int RS = grid_rs(N2);
  constexpr int TPR = PA > PB ? PA : PB;
  static_assert(TPR <= 64 && NTF % 64 == 0, "rows must fit in a wave");
  constexpr int RPW = 64 / TPR;
  constexpr int RPB = RPW * (NTF / 64);
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int nb = (rows + RPB - 1) / RPB;
  for (int b = 0; b < nb; ++b) {            // uniform trip count
    const int row = b * RPB + (t >> 6) * RPW + lane / TPR;
    const int p = lane % TPR;
    const bool in_row = lane < RPW * TPR && row < rows;
    const bool first = in_row && p < PA, second = in_row && p < PB;
    cplx<T>* a = A + (in_row ? row : 0) * RS;
    cplx<T> v[PB];
    if (first) {
#pragma unroll
      for (int q = 0; q < PB; ++q) v[q] = a[p + PA * q];
      dft_reg<T, PB, INV>(v);
      // twiddle exp(s 2 pi i p k / N2); tw[t] = exp(-2 pi i t / N2), p k < N2
#pragma unroll
      for (int k = 1; k < PB; ++k) {
        cplx<T> w = tw[p * k];
        if (INV) w.y = -w.y;
        v[k] = cmul(v[k], w);
      }
    }
    wave_sync();
    if (first) {
#pragma unroll
      for (int k = 0; k < PB; ++k) a[p * PB + (k + p) % PB] = v[k];   // Y[p][k], rotated by p
    }
    wave_sync();
    cplx<T> u[PA];
    if (second) {
#pragma unroll
      for (int q = 0; q < PA; ++q) u[q] = a[q * PB + (p + q) % PB];   // Y[q][k1 = p]
      dft_reg<T, PA, INV>(u);
    }
    wave_sync();
    if (second) {
#pragma unroll
      for (int k2 = 0; k2 < PA; ++k2) a[p + PB * k2] = u[k2];
    }
    wave_sync();
  }
  __syncthreads();
}

// GH[v][r][mode] holds G on entry and H on exit (elements E: complex T, or
// bfloat16 pairs read and written in FP32 arithmetic).  Vs[r][i1][i2] is
// V / (N1 N2) (T).  Work: blockIdx -> ipw consecutive (problem, radius,
// vector) items.
template <typename T, typename E, int N1, int N2, int PA, int PB, int NTF>
__global__ void __launch_bounds__(NTF)
k_angular_grid(E* __restrict__ GH, int nprob, int nvec, int n_r, const DProb* __restrict__ probs,
               const cplx<T>* __restrict__ tw2g, int ipw) {
  constexpr int RS = grid_rs(N2);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);   // [N1][RS]
  cplx<T>* tw = A + N1 * RS;                            // [N2]
  const int64_t per_prob = (int64_t)n_r * nvec;
  const int64_t total = per_prob * nprob;
  const int nwg = (int)((total + ipw - 1) / ipw);
  const int slot = xcd_slot(nwg);
  if (slot >= nwg) return;
  const int t = threadIdx.x;
  for (int i = t; i < N2; i += NTF) tw[i] = tw2g[i];
  const int64_t it0 = (int64_t)slot * ipw;
  const int64_t it1 = total < it0 + ipw ? total : it0 + ipw;
  for (int64_t it = it0; it < it1; ++it) {
    const int pi = (int)(it / per_prob);
    const int rem = (int)(it - pi * per_prob);
    const int r = rem / nvec, v = rem - r * nvec;
    const DProb& pb = probs[pi];
    const int n_modes = pb.n_modes;
    const DMode* modes = pb.modes;
    const T* vr = reinterpret_cast<const T*>(pb.Vs) + (int64_t)r * N1 * N2;
    E* slab = GH + slab_off(pb, nvec, n_r, v, r);
    for (int i = t; i < N1 * RS; i += NTF) A[i] = cplx<T>{(T)0, (T)0};
    __syncthreads();
    for (int i = t; i < n_modes; i += NTF) {
      const int bo = modes[i].boff;   // bin1 * N2 + bin2
      A[(bo / N2) * RS + bo % N2] = eload<T>(slab + i);
    }
    __syncthreads();
    row_dft2<T, N2, PA, PB, NTF, true>(A, N1, tw);
    // theta1: inverse DFT of each column, times V, forward DFT
    for (int j = t; j < N2; j += NTF) {
      cplx<T> c[N1];
#pragma unroll
      for (int i = 0; i < N1; ++i) c[i] = A[i * RS + j];
      dft_reg<T, N1, true>(c);
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const T s = vr[i * N2 + j];
        c[i] = cplx<T>{c[i].x * s, c[i].y * s};
      }
      dft_reg<T, N1, false>(c);
#pragma unroll
      for (int i = 0; i < N1; ++i) A[i * RS + j] = c[i];
    }
    __syncthreads();
    row_dft2<T, N2, PA, PB, NTF, false>(A, N1, tw);
    for (int i = t; i < n_modes; i += NTF) {
      const int bo = modes[i].boff;
      estore(slab + i, A[(bo / N2) * RS + bo % N2]);
    }
    __syncthreads();
  }
}

}  // namespace helic
