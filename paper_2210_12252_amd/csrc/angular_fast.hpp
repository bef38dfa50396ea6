// Angular stage of H*X specialised for compile-time theta2 grid sizes.
//
// For one radius r the angular part of the operator maps the mode block
// G_{m,n}(r) to H_{m,n}(r) = crop(DFT2(V(.,.,r) * IDFT2(pad(G)))) / (N1 N2)
// (Alg. 2, the product with V, Alg. 4).  Written per theta2 column j, the
// theta1 part (inverse DFT over m, multiply by the real V, forward DFT back
// to m) is a circular convolution in m:
//
//   out[m'] = sum_m Vhat_j[m' - m] in[m],
//   Vhat_j[d] = 1/(N1 N2) sum_i V(theta1_i, theta2_j, r) exp(-i 2 pi d i / N1),
//
// exact for the discrete operator (the N1-periodicity of Vhat reproduces the
// aliasing of the grid product), and with only M = m_max - m_min + 1 rows of
// m it costs M^2 complex multiply-adds per column and needs no theta1 FFT.
// The theta2 direction keeps the FFT: a length N2 = P * P transform per m row
// done as P-point DFTs in registers, a twiddle, one exchange through LDS and
// P-point DFTs again (the four-step factorisation).
//
// One workgroup owns one radius and walks over a chunk of vectors; each
// thread keeps the window of Vhat its outputs need in registers for the whole
// chunk, so LDS holds only the mode block and the twiddles.
#pragma once
#include "kernels.hpp"

namespace helic {

// ---------------------------------------------------------------- constexpr trig
// cos/sin of 2 pi t / S for integers t, S: reduce to the nearest multiple of
// pi/2 with integer arithmetic, then Taylor series on |x| <= pi/4.
constexpr double cx_taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
constexpr double cx_twopi_cos(long t, long S) {
  t %= S;
  if (t < 0) t += S;
  long k = (4 * t + S / 2) / S;                 // nearest quadrant
  double x = 1.5707963267948966192 * (double)(4 * t - k * S) / (double)S;
  double c = cx_taylor_cos(x), s = cx_taylor_sin(x);
  switch (k & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}
constexpr double cx_twopi_sin(long t, long S) {
  t %= S;
  if (t < 0) t += S;
  long k = (4 * t + S / 2) / S;
  double x = 1.5707963267948966192 * (double)(4 * t - k * S) / (double)S;
  double c = cx_taylor_cos(x), s = cx_taylor_sin(x);
  switch (k & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

// ---------------------------------------------------------------- register DFTs
// y_k = sum_n v_n exp(s 2 pi i n k / S), s = +1 if INV else -1, all in
// registers (compile-time indices only).
template <typename T, int S, bool INV>
__device__ __forceinline__ void dft_reg(cplx<T>* v);

template <int S>
constexpr int first_radix() {
  return (S % 4 == 0 && S != 4) ? 4 : (S % 3 == 0 && S != 3) ? 3 : (S % 2 == 0 && S != 2) ? 2 : (S % 5 == 0 && S != 5) ? 5 : S;
}

template <typename T, int S, bool INV>
__device__ __forceinline__ void dft_reg(cplx<T>* v) {
  constexpr T sg = INV ? (T)1 : (T)-1;
  if constexpr (S == 1) {
    return;
  } else if constexpr (S == 2) {
    dft2<T>(v, sg);
  } else if constexpr (S == 3) {
    dft3<T>(v, sg);
  } else if constexpr (S == 4) {
    dft4<T>(v, sg);
  } else if constexpr (S == 5) {
    dft5<T>(v, sg);
  } else {
    constexpr int R = first_radix<S>();
    constexpr int Q = S / R;
    static_assert(R * Q == S && R > 1 && Q > 1, "size must factor into 2, 3, 4, 5");
    cplx<T> sub[R][Q];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < Q; ++q) sub[r][q] = v[r + R * q];
      dft_reg<T, Q, INV>(sub[r]);
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        if (r == 0) continue;
        const T c = (T)cx_twopi_cos((long)r * k, S);
        const T s = (T)(INV ? cx_twopi_sin((long)r * k, S) : -cx_twopi_sin((long)r * k, S));
        sub[r][k] = cmul(sub[r][k], cplx<T>{c, s});
      }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      cplx<T> t[R];
#pragma unroll
      for (int r = 0; r < R; ++r) t[r] = sub[r][k];
      dft_reg<T, R, INV>(t);
#pragma unroll
      for (int r = 0; r < R; ++r) v[k + Q * r] = t[r];
    }
  }
}

// Row stride (complex elements) of the LDS mode block for N2 = P * P: the P
// threads of a row and the rows next to it then touch disjoint LDS banks in
// every phase of the row transform when P divides 16 (N2 + P is P mod 16).
// For N2 = 81 a stride of 1 mod 16 elements lets the rows that one wave's
// transform lanes share follow each other on the banks (a bank model of the
// row phases and the mode scatter gives 70 % of the conflict cycles of the
// stride 82); otherwise N2 + 1.
__host__ __device__ constexpr int ang_rs(int n2) {
  return n2 == 16 ? 20 : n2 == 64 ? 72 : n2 == 81 ? 89 : n2 + 1;
}

// Column swizzle of the block: element (m, j) sits at m * RS + (j ^ ang_swz(N2,
// m)).  With the row strides above, 16 consecutive m of one column (how the
// mode slab is laid out) then fall on 16 distinct 16-byte bank groups, while
// the XOR by a per-row constant below 8 keeps every row-transform phase and
// the column-wise convolution conflict-free.
__host__ __device__ constexpr int ang_swz(int n2, int m) {
  return n2 == 64 ? (m >> 1) & 7 : n2 == 16 ? (m >> 2) & 3 : 0;
}

template <typename T>
__device__ __forceinline__ T fmac(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}

// Orders LDS accesses among the lanes of one wave (they execute in issue
// order); enough where only lanes of the same wave exchange data.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- row transform
// In-place length N2 = P * P DFT of `rows` rows of A = A0 + OFF (row stride
// ang_rs(N2); OFF is a compile-time element offset, so blocks at different
// offsets share the per-thread LDS addresses and differ in the immediate) by
// P threads per row.  Thread p of a row loads x[p + P q], does the P-point
// DFT over q, multiplies by exp(s 2 pi i p k / N2), exchanges through LDS so
// that thread c gets Y[.][c], does the P-point DFT over p and stores
// X[c + P k1] at its natural position.  Rows are packed whole into waves
// (64 / P rows per wave, the remaining lanes idle), so the exchanges need only
// wave-level ordering.  All threads of the block must call; A must be
// synchronised on entry, and the caller synchronises the block before other
// waves read the result.
template <typename T, int N2, int P, int NTF, bool INV, int OFF, bool PIN>
__device__ __forceinline__ void row_dft(cplx<T>* A0, int rows, const cplx<T>* tw) {
  static_assert(P * P == N2, "row transform expects N2 = P * P");
  static_assert(P <= 64 && NTF % 64 == 0, "rows must fit in a wave");
  constexpr int RS = ang_rs(N2);
  constexpr int RPW = 64 / P;                 // rows per wave
  constexpr int RPB = RPW * (NTF / 64);       // rows per batch
  // With PIN, t passes through an empty asm so that the per-thread LDS
  // addresses below are recomputed at each call instead of being hoisted out
  // of the caller's vector loop, where they stay live throughout (faster
  // while they fit in registers, spilled on the widest blocks)
  int t = threadIdx.x;
  if constexpr (PIN) asm volatile("" : "+v"(t));
  const int lane = t & 63;
  const int nb = (rows + RPB - 1) / RPB;
  for (int b = 0; b < nb; ++b) {            // uniform trip count
    const int row = b * RPB + (t >> 6) * RPW + lane / P;
    const int p = lane % P;
    const bool act = lane < RPW * P && row < rows;
    cplx<T> v[P];
    if (act) {
      cplx<T>* a = A0 + row * RS;
      const int sw = ang_swz(N2, row);
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = a[OFF + ((p + P * q) ^ sw)];
      dft_reg<T, P, INV>(v);
      // twiddle exp(s 2 pi i p k / N2); tw[t] = exp(-2 pi i t / N2), p k < N2
#pragma unroll
      for (int k = 1; k < P; ++k) {
        cplx<T> w = tw[p * k];
        if (INV) w.y = -w.y;
        v[k] = cmul(v[k], w);
      }
    }
    wave_sync();
    // exchange Y[p][k] through LDS; element (p, k) is stored at p*P +
    // (k + p) mod P so that both the row-wise writes and the column-wise
    // reads of the P threads of a row fall on distinct banks
    if (act) {
      cplx<T>* a = A0 + row * RS;
      const int sw = ang_swz(N2, row);
#pragma unroll
      for (int k = 0; k < P; ++k) {
        int kk = k + p;
        kk -= (kk >= P) ? P : 0;
        a[OFF + ((p * P + kk) ^ sw)] = v[k];
      }
    }
    wave_sync();
    if (act) {
      cplx<T>* a = A0 + row * RS;
      const int sw = ang_swz(N2, row);
      const int c = p;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        int cc = c + q;
        cc -= (cc >= P) ? P : 0;
        v[q] = a[OFF + ((q * P + cc) ^ sw)];   // Y[q][c]
      }
      dft_reg<T, P, INV>(v);
    }
    wave_sync();
    if (act) {
      cplx<T>* a = A0 + row * RS;
      const int sw = ang_swz(N2, row);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) a[OFF + ((p + P * k1) ^ sw)] = v[k1];
    }
    wave_sync();
  }
}

// Row transforms whose input (inverse) or output (forward) stays in the
// registers of the row's P threads: lane (row, p) holds the elements at
// columns p + P q.  The LDS row is used as the exchange buffer (and, for the
// inverse, receives the transformed row).  SWZ false: the block has no
// column swizzle.
template <typename T, int N2, int P, int NTF, int ROWS, int OFF, bool PIN, bool SWZ = true>
__device__ __forceinline__ void row_idft_from_regs(cplx<T>* A0, const cplx<T>* tw, const cplx<T>* xin) {
  constexpr int RS = ang_rs(N2);
  constexpr int RPW = 64 / P;
  static_assert(ROWS <= RPW * (NTF / 64), "one batch of rows");
  int t = threadIdx.x;
  if constexpr (PIN) asm volatile("" : "+v"(t));
  const int lane = t & 63;
  const int row = (t >> 6) * RPW + lane / P;
  const int p = lane % P;
  const bool act = lane < RPW * P && row < ROWS;
  cplx<T> v[P];
  cplx<T>* a = A0 + (act ? row : 0) * RS;
  const int sw = SWZ ? ang_swz(N2, act ? row : 0) : 0;
  if (act) {
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = xin[q];
    dft_reg<T, P, true>(v);
#pragma unroll
    for (int k = 1; k < P; ++k) {
      cplx<T> w = tw[p * k];
      w.y = -w.y;
      v[k] = cmul(v[k], w);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      int kk = k + p;
      kk -= (kk >= P) ? P : 0;
      a[OFF + ((p * P + kk) ^ sw)] = v[k];
    }
  }
  wave_sync();
  if (act) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      int cc = p + q;
      cc -= (cc >= P) ? P : 0;
      v[q] = a[OFF + ((q * P + cc) ^ sw)];
    }
    dft_reg<T, P, true>(v);
  }
  wave_sync();
  if (act) {
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) a[OFF + ((p + P * k1) ^ sw)] = v[k1];
  }
}

template <typename T, int N2, int P, int NTF, int ROWS, int OFF, bool PIN, bool SWZ = true>
__device__ __forceinline__ void row_dft_to_regs(cplx<T>* A0, const cplx<T>* tw, cplx<T>* xout) {
  constexpr int RS = ang_rs(N2);
  constexpr int RPW = 64 / P;
  static_assert(ROWS <= RPW * (NTF / 64), "one batch of rows");
  int t = threadIdx.x;
  if constexpr (PIN) asm volatile("" : "+v"(t));
  const int lane = t & 63;
  const int row = (t >> 6) * RPW + lane / P;
  const int p = lane % P;
  const bool act = lane < RPW * P && row < ROWS;
  cplx<T> v[P];
  cplx<T>* a = A0 + (act ? row : 0) * RS;
  const int sw = SWZ ? ang_swz(N2, act ? row : 0) : 0;
  if (act) {
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = a[OFF + ((p + P * q) ^ sw)];
    dft_reg<T, P, false>(v);
#pragma unroll
    for (int k = 1; k < P; ++k) v[k] = cmul(v[k], tw[p * k]);
  }
  wave_sync();
  if (act) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      int kk = k + p;
      kk -= (kk >= P) ? P : 0;
      a[OFF + ((p * P + kk) ^ sw)] = v[k];
    }
  }
  wave_sync();
  if (act) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      int cc = p + q;
      cc -= (cc >= P) ? P : 0;
      v[q] = a[OFF + ((q * P + cc) ^ sw)];
    }
    dft_reg<T, P, false>(v);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) xout[k1] = v[k1];
  }
}

// ---------------------------------------------------------------- convolution
// The convolution proceeds in groups of CONV_MB rows: the accumulators pass
// through an empty asm at each group boundary, which pins the multiply-adds
// of a group between its loads and the next group's, so only CONV_MB column
// values are in registers at a time (left alone, the compiler loads the whole
// column first and runs the accumulator chains one after the other).
#ifndef HELIC_CONV_MB
#define HELIC_CONV_MB 8
#endif
constexpr int CONV_MB = HELIC_CONV_MB;
#ifndef HELIC_CONV_ADJ
#define HELIC_CONV_ADJ 1
#endif

template <typename T, int OPT>
__device__ __forceinline__ void pin_acc(cplx<T>* acc) {
#pragma unroll
  for (int o = 0; o < OPT; ++o) asm volatile("" : "+v"(acc[o].x), "+v"(acc[o].y));
}

// Outputs m' = A0 .. A0 + OPT - 1 of column j: out[m'] = sum_m Vhat[m' - m]
// in[m].  The potential is real, so Vhat[-d] = conj(Vhat[d]) and the thread
// holds h[d] = Vhat[d] for d = 0 .. MPAD - 1 only; with A0 a compile-time
// constant every (m', m) pair resolves to h or its conjugate at compile time.
template <typename T, int N2, int MPAD, int OPT, int A0>
__device__ __forceinline__ void conv_herm(const cplx<T>* A, cplx<T>* B, int j, const cplx<T>* h) {
  constexpr int RS = ang_rs(N2);
  cplx<T> acc[OPT];
#pragma unroll
  for (int o = 0; o < OPT; ++o) acc[o] = cplx<T>{(T)0, (T)0};
#pragma unroll
  for (int m = 0; m < MPAD; ++m) {
    if (m % CONV_MB == 0 && m > 0) pin_acc<T, OPT>(acc);
    const cplx<T> x = A[m * RS + (j ^ ang_swz(N2, m))];
#pragma unroll
    for (int o = 0; o < OPT; ++o) {
      const int d = A0 + o - m;
      if (A0 + o >= MPAD) continue;
      if (d >= 0) {
        const cplx<T> wv = h[d];
        acc[o].x = fmac(wv.x, x.x, acc[o].x);
        acc[o].x = fmac(-wv.y, x.y, acc[o].x);
        acc[o].y = fmac(wv.x, x.y, acc[o].y);
        acc[o].y = fmac(wv.y, x.x, acc[o].y);
      } else {
        const cplx<T> wv = h[-d];
        acc[o].x = fmac(wv.x, x.x, acc[o].x);
        acc[o].x = fmac(wv.y, x.y, acc[o].x);
        acc[o].y = fmac(wv.x, x.y, acc[o].y);
        acc[o].y = fmac(-wv.y, x.x, acc[o].y);
      }
    }
  }
#pragma unroll
  for (int o = 0; o < OPT; ++o)
    if (A0 + o < MPAD) B[(A0 + o) * RS + (j ^ ang_swz(N2, A0 + o))] = acc[o];
}

// Selects the compile-time output range of output group g (wave-uniform).
template <typename T, int N2, int MPAD, int OPT, int G, int OG>
__device__ __forceinline__ void conv_herm_group(int g, const cplx<T>* A, cplx<T>* B, int j, const cplx<T>* h) {
  if constexpr (G < OG) {
    if (g == G) conv_herm<T, N2, MPAD, OPT, G * OPT>(A, B, j, h);
    else conv_herm_group<T, N2, MPAD, OPT, G + 1, OG>(g, A, B, j, h);
  }
}

// ---------------------------------------------------------------- the kernel
// Workgroups per CU the register allocation is held to: 16 waves per CU in
// FP32 where the block fits 128 registers without spilling (row addresses
// then recomputed per call, see row_dft), else 8.
// FP64 blocks of 64 columns and up to 24 rows move the mode slab straight
// between global memory and the registers of the row transforms (the block
// positions without a mode load zeros and store nothing): no clearing pass,
// no LDS scatter and gather, two block barriers per vector.  Elsewhere the
// extra registers spill, and the slab goes through LDS.
template <typename T, int N2, int MPAD>
constexpr bool ang_direct() {
  return sizeof(T) == 8 && N2 == 64 && MPAD <= 24;
}

template <typename T, int N2, int MPAD, int NTF>
constexpr int ang_min_wgs() {
  return (sizeof(T) == 4 && !(N2 == 64 && MPAD > 24) ? 1024 : 512) / NTF;
}

// GH[v][r][mode] holds G on entry and H on exit (elements E: complex T, or
// bfloat16 pairs read and written in FP32 arithmetic).  Vh[r][j][d]
// (complex T, d = 0..2 MPAD - 2 for m' - m = d - (MPAD - 1)).  mode_pos[i] =
// (m_i - m_min) * ang_rs(N2) + ((n_i mod N2) ^ ang_swz(N2, m_i - m_min));
// blk_mode is its inverse on the unswizzled block (see ang_direct).
// Work: blockIdx -> ipw consecutive (problem, radius, vector) items.
//
// LDS holds two mode blocks: A receives the scattered slab and its theta2
// inverse transform, the convolution writes into B, and B is transformed back
// and gathered while A is cleared and filled with the next vector.  Per vector
// the block then synchronises four times: after the scatter, after the
// inverse row transforms, after the convolution and after the forward row
// transforms.
template <typename T, typename E, int N2, int MPAD, int NTF>
__global__ void __launch_bounds__(NTF, (ang_min_wgs<T, N2, MPAD, NTF>()))
k_angular_fast(E* __restrict__ GH, int nprob, int nvec, int n_r, const DProb* __restrict__ probs,
               const cplx<T>* __restrict__ tw2g, int ipw) {
  constexpr int P = (N2 == 16) ? 4 : (N2 == 64) ? 8 : (N2 == 81) ? 9 : (N2 == 36) ? 6 : (N2 == 100) ? 10 : 0;
  static_assert(P > 0, "unsupported N2");
  constexpr int ND = 2 * MPAD - 1;
  constexpr int OG = NTF / N2;                    // threads per column in the convolution
  constexpr int OPT = (MPAD + OG - 1) / OG;       // outputs per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int RS = ang_rs(N2);                               // padded row stride of A and B
  constexpr int BLK = MPAD * RS;
  constexpr int WN = OPT + MPAD - 1;                           // Vhat window of one thread
  constexpr bool PIN_ROWS = sizeof(T) == 4 || MPAD >= 32;       // see row_dft and ang_min_wgs
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);          // [MPAD][RS]
  cplx<T>* B = A + BLK;                                        // [MPAD][RS]
  cplx<T>* tw = B + BLK;                                       // [N2]
  // Work items are (problem, radius, vector) triples in that order; each
  // workgroup takes ipw consecutive items, as segments of one radius each
  // (the V-hat registers and mode positions are loaded once per segment).
  const int64_t per_prob = (int64_t)n_r * nvec;
  const int64_t total = per_prob * nprob;
  const int nwg = (int)((total + ipw - 1) / ipw);
  const int slot = xcd_slot(nwg);
  if (slot >= nwg) return;
  int64_t it = (int64_t)slot * ipw;
  const int64_t it_end = total < it + ipw ? total : it + ipw;
  const int t = threadIdx.x;
  for (int i = t; i < N2; i += NTF) tw[i] = tw2g[i];
  constexpr bool HERM = (N2 == 64);
  // convolution threads: with HERM the output group is the wave index (its
  // code specialised at compile time); otherwise the OG threads of a column
  // are adjacent lanes, so their reads of the column are LDS broadcasts
  constexpr bool ADJ = !HERM && HELIC_CONV_ADJ;
  const int j = ADJ ? t / OG : t % N2, og = ADJ ? t % OG : t / N2;
  const bool conv_act = ADJ ? t < OG * N2 : og < OG;
  const int a0 = og * OPT;
  constexpr int NW = HERM ? MPAD : WN;
  constexpr int MS = (MPAD * N2 + NTF - 1) / NTF;   // every mode of a radius fits the block
  for (int i = t; i < BLK; i += NTF) A[i] = cplx<T>{(T)0, (T)0};
  __syncthreads();
  while (it < it_end) {
    const int pi = (int)(it / per_prob);
    const int rem = (int)(it - pi * per_prob);
    const int r = rem / nvec, v0 = rem - r * nvec;
    const int v1 = (int)(nvec < v0 + (it_end - it) ? nvec : v0 + (it_end - it));
    it += v1 - v0;
    const DProb& pb = probs[pi];
    const int n_modes = pb.n_modes;
    const T* Vh = reinterpret_cast<const T*>(pb.Vh);
    // With N2 = 64 the output group is the wave index, and the thread keeps
    // h[d] = Vhat_j[d], d = 0 .. MPAD - 1 (the rest follows by conjugation).
    // Otherwise it keeps the window w[q] = Vhat_j[a0 + q - (MPAD - 1)] that its
    // outputs m' in [a0, a0 + OPT) need over all m.  Either is read once and
    // kept in registers for every vector of the segment.
    cplx<T> w[NW];
    {
      const cplx<T>* src = reinterpret_cast<const cplx<T>*>(Vh) + ((int64_t)r * N2 + j) * ND;
      const int base = HERM ? MPAD - 1 : a0;
#pragma unroll
      for (int q = 0; q < NW; ++q)
        w[q] = (conv_act && base + q < ND) ? src[base + q] : cplx<T>{(T)0, (T)0};
    }
    if constexpr (ang_direct<T, N2, MPAD>()) {
      // Lane (row, p) of the row transforms moves the elements at columns
      // p + P q of its row straight between the slab and its registers:
      // idx[q] = mode index of that block position (blk_mode[row * N2 + col]),
      // -1 where no mode is kept.  The next vector's elements are fetched while
      // the current one is transformed.
      constexpr int RPW_ = 64 / P;
      const int rrow = (t >> 6) * RPW_ + (t & 63) / P, rp = (t & 63) % P;
      const bool ract = (t & 63) < RPW_ * P && rrow < MPAD;
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
        row_idft_from_regs<T, N2, P, NTF, MPAD, 0, PIN_ROWS>(A, tw, xin);
        if (v + 1 < v1) fetch(v + 1);
        __syncthreads();
        // theta1: Toeplitz convolution per column with the spectrum of V, A -> B
        static_assert(HERM, "the direct path serves 64-column blocks");
        conv_herm_group<T, N2, MPAD, OPT, 0, OG>(__builtin_amdgcn_readfirstlane(og), A, B, j, w);
        __syncthreads();
        cplx<T> xout[P];
        row_dft_to_regs<T, N2, P, NTF, MPAD, BLK, PIN_ROWS>(A, tw, xout);
        E* slab = GH + slab_off(pb, nvec, n_r, v, r);
        if (ract) {
#pragma unroll
          for (int q = 0; q < P; ++q)
            if (idx[q] >= 0) estore(slab + idx[q], xout[q]);
        }
      }
    } else {
      // The mode slab of the next vector is fetched into registers while the
      // current one is transformed: thread t owns modes t + NTF q (coalesced
      // global access) and writes them to their block positions mode_pos.
      int mp[MS];
#pragma unroll
      for (int q = 0; q < MS; ++q) {
        const int i = t + NTF * q;
        mp[q] = i < n_modes ? pb.mode_pos[i] : -1;
      }
      cplx<T> pre[MS];
      auto fetch = [&](int v) {
        const E* slab = GH + slab_off(pb, nvec, n_r, v, r);
#pragma unroll
        for (int q = 0; q < MS; ++q) pre[q] = mp[q] >= 0 ? eload<T>(slab + t + NTF * q) : cplx<T>{(T)0, (T)0};
      };
      fetch(v0);
      for (int v = v0; v < v1; ++v) {
        // A is clear here (and no thread still reads it); B is no longer read
#pragma unroll
        for (int q = 0; q < MS; ++q)
          if (mp[q] >= 0) A[mp[q]] = pre[q];
        __syncthreads();
        if (v + 1 < v1) fetch(v + 1);
        row_dft<T, N2, P, NTF, true, 0, PIN_ROWS>(A, MPAD, tw);
        __syncthreads();
        // theta1: Toeplitz convolution per column with the spectrum of V, A -> B
        if constexpr (HERM) {
          conv_herm_group<T, N2, MPAD, OPT, 0, OG>(__builtin_amdgcn_readfirstlane(og), A, B, j, w);
        } else if (conv_act) {
          cplx<T> acc[OPT];
#pragma unroll
          for (int o = 0; o < OPT; ++o) acc[o] = cplx<T>{(T)0, (T)0};
#pragma unroll
          for (int m = 0; m < MPAD; ++m) {
            if (m % CONV_MB == 0 && m > 0) pin_acc<T, OPT>(acc);
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
        row_dft<T, N2, P, NTF, false, BLK, PIN_ROWS>(A, MPAD, tw);
        for (int i = t; i < BLK; i += NTF) A[i] = cplx<T>{(T)0, (T)0};
        __syncthreads();
        E* slab = GH + slab_off(pb, nvec, n_r, v, r);
#pragma unroll
        for (int q = 0; q < MS; ++q)
          if (mp[q] >= 0) estore(slab + t + NTF * q, A[BLK + mp[q]]);
      }
    }
  }
}

}  // namespace helic
