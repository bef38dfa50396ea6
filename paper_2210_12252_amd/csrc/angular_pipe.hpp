// Angular stage of H*X by the theta1 convolution of k_angular_fast, with the
// workgroup's waves split into two roles that work on different vectors.
//
// Per radius and vector it computes exactly what k_angular_fast computes
// (Alg. 2, the product with V as the circular convolution
// out[m'] = sum_m Vhat_j[m' - m] in[m] per theta2 column j, Alg. 4).  There
// all waves take one vector through scatter, theta2 inverse rows,
// convolution, theta2 forward rows and gather, with four block barriers per
// vector, and on blocks whose rows fit in half the waves the other half idles
// through both row phases.
//
// Here the first half of the waves (row waves) does only the theta2 row
// transforms, moving the slab straight between global memory and its
// registers (lane (row, p) holds block positions p + P q; no LDS scatter,
// gather or clearing), and the second half (convolution waves, the OG
// threads of a column on adjacent lanes) does only the convolution.  LDS
// holds two A blocks (inverse rows' output) and two B blocks (convolution
// output), laid out (row stride, column swizzle) as in k_angular_fast.  In
// step s of a radius segment the row waves run the inverse rows of vector s
// (slab -> A[s % 2], the next vector's slab fetched behind them) and the
// forward rows of vector s - 2 (B[s % 2] -> slab), while the convolution
// waves run vector s - 1 (A[(s - 1) % 2] -> B[(s - 1) % 2]); one block
// barrier closes a step, and a segment of n vectors takes n + 2 steps.  On
// each SIMD a row wave and a convolution wave then share the issue slots.
#pragma once

#include "angular_fast.hpp"

namespace helic {

// Rows of the convolution between accumulator pins (see CONV_MB).
#ifndef HELIC_PIPE_MB
#define HELIC_PIPE_MB 4
#endif
constexpr int PIPE_MB = HELIC_PIPE_MB;

template <int N2>
constexpr int pipe_p() {
  return N2 == 16 ? 4 : N2 == 64 ? 8 : N2 == 81 ? 9 : N2 == 36 ? 6 : N2 == 100 ? 10 : 0;
}

// The rows of a block must fit one pass of the row waves (half the block).
template <int N2, int MPAD, int NTF>
constexpr bool pipe_fits() {
  return pipe_p<N2>() > 0 && (64 / pipe_p<N2>()) * (NTF / 128) >= MPAD && NTF % 128 == 0;
}

// GH, probs, tw2g, ipw as for k_angular_fast (blk_mode and the V-hat
// layout are the same).  LDS: four blocks of MPAD x ang_rs(N2) and the N2
// twiddles.
template <typename T, typename E, int N2, int MPAD, int NTF>
__global__ void __launch_bounds__(NTF, 1)
k_angular_pipe(E* __restrict__ GH, int nprob, int nvec, int n_r, const DProb* __restrict__ probs,
               const cplx<T>* __restrict__ tw2g, int ipw) {
  constexpr int P = pipe_p<N2>();
  static_assert(pipe_fits<N2, MPAD, NTF>(), "rows must fit the row waves");
  static_assert(sizeof(T) == 8, "mode indices are packed into FP64 registers");
  constexpr int NR = NTF / 2;                     // row-transform threads; the rest convolve
  constexpr int RPW = 64 / P;
  constexpr int ND = 2 * MPAD - 1;
  constexpr int OG = NR / N2;                     // convolution threads per column
  static_assert(OG >= 1, "a column per convolution thread at least");
  constexpr int OPT = (MPAD + OG - 1) / OG;       // outputs per convolution thread
  constexpr int RS = ang_rs(N2);
  constexpr int BLK = MPAD * RS;
  // With one output group per convolution wave (a column per lane: N2 = 64
  // and four groups) the group's code is specialised at compile time and,
  // V being real (Vhat_j[-d] = conj Vhat_j[d]), the thread holds
  // Vhat_j[d], d = 0 .. MPAD - 1 only, as in k_angular_fast; otherwise the
  // window w[q] = Vhat_j[a0 + q - (MPAD - 1)] of its outputs.
  constexpr bool HERM = (N2 == 64 && OG * 64 == NR);
  constexpr int WN = HERM ? MPAD : OPT + MPAD - 1;   // Vhat registers of one convolution thread
  static_assert(WN >= P + (P + 3) / 4, "the row waves' registers fit the window");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* const Ab = reinterpret_cast<cplx<T>*>(smem_raw);   // A[0], A[1]
  cplx<T>* const Bb = Ab + 2 * BLK;                           // B[0], B[1]
  cplx<T>* const tw = Bb + 2 * BLK;                           // [N2]
  const int64_t per_prob = (int64_t)n_r * nvec;
  const int64_t total = per_prob * nprob;
  const int nwg = (int)((total + ipw - 1) / ipw);
  const int slot = xcd_slot(nwg);
  if (slot >= nwg) return;
  int64_t it = (int64_t)slot * ipw;
  const int64_t it_end = total < it + ipw ? total : it + ipw;
  const int t = threadIdx.x;
  for (int i = t; i < N2; i += NTF) tw[i] = tw2g[i];
  const bool row_role = t < NR;
  // row waves: lane (row, p) moves the block positions p + P q of its row
  const int lane = t & 63;
  const int rrow = (t >> 6) * RPW + lane / P, rp = lane % P;
  const bool ract = row_role && lane < RPW * P && rrow < MPAD;
  // convolution waves: the OG threads of a column are adjacent lanes (their
  // reads of the column are LDS broadcasts)
  const int c = t - NR;
  const int j = row_role ? 0 : HERM ? (c & 63) : c / OG;
  const int og = row_role ? 0 : HERM ? (c >> 6) : c % OG;
  const bool conv_act = !row_role && c < OG * N2;
  const int a0 = og * OPT;
  __syncthreads();
  while (it < it_end) {
    const int pi = (int)(it / per_prob);
    const int rem = (int)(it - pi * per_prob);
    const int r = rem / nvec, v0 = rem - r * nvec;
    const int v1 = (int)(nvec < v0 + (it_end - it) ? nvec : v0 + (it_end - it));
    it += v1 - v0;
    const int nv = v1 - v0;
    const DProb& pb = probs[pi];
    // One register array serves both roles (each lives through the whole
    // step loop, and the two together would not fit): for the convolution
    // waves the window w[q] = Vhat_j[a0 + q - (MPAD - 1)] of the thread's
    // outputs; for the row waves the next vector's slab values at the
    // lane's block positions (w[0 .. P - 1]) and those positions' mode
    // indices, -1 where none (packed four to an element from w[P] on).
    cplx<T> w[WN];
    auto idx = [&](int q) -> int {
      const T d = (q & 2) ? w[P + q / 4].y : w[P + q / 4].x;
      return (q & 1) ? __double2hiint(d) : __double2loint(d);
    };
    auto fetch = [&](int v) {
      const E* slab = GH + slab_off(pb, nvec, n_r, v, r);
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int i = idx(q);
        w[q] = i >= 0 ? eload<T>(slab + i) : cplx<T>{(T)0, (T)0};
      }
    };
    if (row_role) {
      int id[4 * ((P + 3) / 4)];
#pragma unroll
      for (int q = 0; q < 4 * ((P + 3) / 4); ++q) id[q] = ract && q < P ? pb.blk_mode[rrow * N2 + rp + P * q] : -1;
#pragma unroll
      for (int g = 0; g < (P + 3) / 4; ++g)
        w[P + g] = cplx<T>{__hiloint2double(id[4 * g + 1], id[4 * g]), __hiloint2double(id[4 * g + 3], id[4 * g + 2])};
      fetch(v0);
    } else {
      const cplx<T>* src = reinterpret_cast<const cplx<T>*>(pb.Vh) + ((int64_t)r * N2 + j) * ND;
      const int base = HERM ? MPAD - 1 : a0;
#pragma unroll
      for (int q = 0; q < WN; ++q) w[q] = (conv_act && base + q < ND) ? src[base + q] : cplx<T>{(T)0, (T)0};
    }
    // step s: row waves take vector s through the inverse rows (slab ->
    // A[s % 2]) and vector s - 2 through the forward rows (B[s % 2] ->
    // slab); convolution waves take vector s - 1 (A[(s - 1) % 2] ->
    // B[(s - 1) % 2]); one block barrier closes the step
    for (int s = 0; s < nv + 2; ++s) {
      if (row_role) {
        // the mode indices pass through an empty asm, so the slab offsets
        // are recomputed where they are used instead of being hoisted out of
        // the loop (they would not fit in registers there)
#pragma unroll
        for (int g = 0; g < (P + 3) / 4; ++g) asm volatile("" : "+v"(w[P + g].x), "+v"(w[P + g].y));
        if (s < nv) {
          row_idft_from_regs<T, N2, P, NR, MPAD, 0, true, true>(Ab + (s & 1) * BLK, tw, w);
          if (s + 1 < nv) fetch(v0 + s + 1);
        }
        if (s >= 2) {
          cplx<T> xout[P];
          row_dft_to_regs<T, N2, P, NR, MPAD, 0, true, true>(Bb + (s & 1) * BLK, tw, xout);
          if (ract) {
            E* slab = GH + slab_off(pb, nvec, n_r, v0 + s - 2, r);
#pragma unroll
            for (int q = 0; q < P; ++q)
              if (idx(q) >= 0) estore(slab + idx(q), xout[q]);
          }
        }
      } else if (HERM && s >= 1 && s <= nv) {
        conv_herm_group<T, N2, MPAD, OPT, 0, OG>(__builtin_amdgcn_readfirstlane(og), Ab + ((s - 1) & 1) * BLK,
                                                 Bb + ((s - 1) & 1) * BLK, j, w);
      } else if (!HERM && conv_act && s >= 1 && s <= nv) {
        const cplx<T>* A = Ab + ((s - 1) & 1) * BLK;
        cplx<T>* B = Bb + ((s - 1) & 1) * BLK;
        cplx<T> acc[OPT];
#pragma unroll
        for (int o = 0; o < OPT; ++o) acc[o] = cplx<T>{(T)0, (T)0};
#pragma unroll
        for (int m = 0; m < MPAD; ++m) {
          if (m % PIPE_MB == 0 && m > 0) pin_acc<T, OPT>(acc);
          const cplx<T> x = A[m * RS + (j ^ ang_swz(N2, m))];
#pragma unroll
          for (int o = 0; o < OPT; ++o) {
            const cplx<T> wv = w[o - m + MPAD - 1];
            acc[o].x = fmac(wv.x, x.x, acc[o].x);
            acc[o].x = fmac(-wv.y, x.y, acc[o].x);
            acc[o].y = fmac(wv.x, x.y, acc[o].y);
            acc[o].y = fmac(wv.y, x.x, acc[o].y);
          }
        }
#pragma unroll
        for (int o = 0; o < OPT; ++o)
          if (a0 + o < MPAD) B[(a0 + o) * RS + (j ^ ang_swz(N2, a0 + o))] = acc[o];
      }
      __syncthreads();
    }
  }
}

}  // namespace helic
