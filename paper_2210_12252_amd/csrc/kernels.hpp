// HIP kernels of the helical-wave Hamiltonian apply on gfx950 (CDNA4).
//
// Data layout in HBM
//   X, Y       coefficient blocks, complex double, column-major (ld >= L), rows
//              in the compact order: grouped by |n|, then sign of n, then m,
//              then k = 1..K (so one group's rows are contiguous).
//   GH         per-(vector, radius) slabs of angular-mode values,
//              GH[v][r][mode] complex T, modes in compact order.  K-inv writes
//              G into it, K-ang overwrites each slab in place with H, K-fwd
//              reads H.
//   Vs         the potential re-laid out per radius, Vs[r][i1][i2], already
//              divided by n_t1 * n_t2 (the forward DFT normalisation).
//   tinv/tfwd  radial tables per |n| group in MFMA fragment order.
//
// Kernels
//   k_radial_inverse   G_{mn}(r_l) = sum_k xi_{|n|,k}(r_l) x_{mnk}   (Alg. 1,
//                      radial part): one |n| group x one vector per
//                      workgroup, a real (n_r x K) by (K x 2 modes) GEMM on
//                      16x16x4 MFMA tiles.
//   k_angular          per (vector, radius) slab in LDS: inverse 2D DFT of the
//                      mode block (Alg. 2), multiply by V, forward 2D DFT and
//                      crop back to the kept modes (Alg. 4); Stockham radix
//                      2/3/4/5 passes through LDS, the theta2 passes only on
//                      the theta1 bins that hold modes, V fused into the
//                      loads of the first forward pass.
//   k_radial_forward   y_{mnk} = kappa x_{mnk} + 2 pi tau sum_l omega_l
//                      xi_{|n|,k}(r_l) H_{mn}(r_l)   (Alg. 3 radial part and
//                      the diagonal terms of Alg. 5): a (K x n_r) by
//                      (n_r x 2 modes) GEMM with the kinetic term in the
//                      epilogue.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace helic {

constexpr int NT = 256;             // threads per workgroup in every kernel
constexpr int MAXGRID = 8192;       // n_t1 * n_t2 bound of k_angular
constexpr int KS_MAX = 24;          // K <= 96 per |n| group
constexpr int FWD_RCHUNK = 32;
constexpr int FWD_PF_RC = 16;       // radii per chunk of the pipelined radial forward kernel
constexpr int FWD_PF_COLS = 256;    // widest staged group (columns) it supports
constexpr int FWD_PF_KT = 6;        // k tiles (of 16) per group it supports
// LDS row stride (elements) of a staged radial tile of colpad columns
// (colpad a multiple of 16): congruent to 16 mod 32, so that the four rows an
// MFMA B operand reads (16 lanes each) fall on disjoint bank ranges.
__host__ __device__ constexpr int lds_stride(int colpad) { return (colpad & 16) ? colpad : colpad + 16; }      // radii staged per LDS round in k_radial_forward

struct DGroup {
  int32_t mode0, nmodes, Kmax, prob;   // modes relative to the problem; prob indexes DProb
  int64_t row0, nrows, tinv_off, tfwd_off;
  int64_t tinv16_off, tfwd16_off;      // offsets (4-element BF16 fragments) of the BF16 tables
};

struct DMode {
  int64_t row0;
  int32_t K;
  int32_t boff;   // LDS offset bin1 * n_t2 + bin2 of the mode in a slab
};

// One problem (basis + potential) of a launch.  A launch covers one problem
// (leading dimensions given by the caller) or a batch of problems whose
// blocks are concatenated: problem p's nvec columns of L_p rows start at
// complex offset nvec * Lpre_p, and its slabs at nvec * n_r * mpre_p.
// Table and potential pointers are in the launch's precision.
struct DProb {
  const DGroup* groups;
  const DMode* modes;
  const int32_t* row_ck;
  const double* kappa;
  const void* tinv;
  const void* tfwd;
  const void* Vs;
  const void* Vh;
  const int32_t* mode_pos;    // mode -> LDS position in the angular block (specialised kernel)
  const int32_t* blk_mode;    // block position (m - m_min) * n_t2 + (n mod n_t2) -> mode, -1 if none
  int64_t Lpre, L, mpre;
  int32_t n_modes, pad;
};

// complex offset of column v of problem pb: ld >= 0 for a single problem,
// ld < 0 for the concatenated batch layout
__device__ __forceinline__ int64_t col_off(const DProb& pb, int64_t ld, int nvec, int v) {
  return ld >= 0 ? (int64_t)v * ld : (int64_t)nvec * pb.Lpre + (int64_t)v * pb.L;
}
__device__ __forceinline__ int64_t slab_off(const DProb& pb, int nvec, int n_r, int v, int r) {
  return (int64_t)nvec * n_r * pb.mpre + ((int64_t)v * n_r + r) * pb.n_modes;
}

struct FftPlan {
  int32_t n, nf;
  int32_t f[12];
};

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by +i (s = +1) or -i (s = -1)
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a, T s) { return {-s * a.y, s * a.x}; }

// Two consecutive elements moved by one memory instruction (16 bytes in FP64).
template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double2 type; };
template <> struct Vec2<float> { typedef float2 type; };

// ---------------------------------------------------------------- BF16 storage
// A complex value stored as two bfloat16 (re in the low half, im in the high
// half of one 32-bit word): the intermediate slabs of the BF16 mode.
struct bf16x2 {
  uint32_t u;
};
// float -> bfloat16 bits, rounded to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

// Slab element E (cplx<double>, cplx<float> or bf16x2) read and written in
// the arithmetic type T of the kernel that moves it.
template <typename T, typename E>
__device__ __forceinline__ cplx<T> eload(const E* p) {
  if constexpr (std::is_same<E, bf16x2>::value) {
    const uint32_t u = p->u;
    return cplx<T>{(T)bf16_lo(u), (T)bf16_hi(u)};
  } else {
    const E e = *p;
    return cplx<T>{(T)e.x, (T)e.y};
  }
}
template <typename T, typename E>
__device__ __forceinline__ void estore(E* p, cplx<T> v) {
  if constexpr (std::is_same<E, bf16x2>::value) {
    p->u = bf16_bits((float)v.x) | (bf16_bits((float)v.y) << 16);
  } else {
    *p = E{v.x, v.y};
  }
}

// 16x16x16 BF16 MFMA with FP32 accumulation: lane l supplies A[l % 16][4 (l /
// 16) + j] and B[4 (l / 16) + j][l % 16] (j = 0..3, four bfloat16 in 64 bits);
// accumulator element i of lane l is D[4 (l / 16) + i][l % 16] (as the 32-bit
// 16x16x4 form).
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4_t mfma_bf16(uint64_t a, uint64_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4_t, a), __builtin_bit_cast(bf16x4_t, b),
                                                   c, 0, 0, 0);
}

template <typename T> struct Mfma;
// 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element i of lane l is D[row(l, i)][l % 16].  The row map
// differs between the 64-bit and the 32-bit forms (checked on gfx950).
template <> struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <> struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// Work item of an XCD-aware launch: workgroups are dealt round-robin to the 8
// XCDs, so consecutive slots of one XCD are given contiguous work indices
// (and share tables or potential slabs in that XCD's L2).
__device__ __forceinline__ int xcd_slot(int nwork) {
  const int per = (nwork + 7) / 8;
  return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// (vector, group) of a workgroup of the radial stages, false if idle.
// order 0: vector-major slots (each XCD runs every group of a few vectors);
// order 1: XCD x takes vectors [x vpx, (x + 1) vpx), vpx = ceil(nvec / 8),
// and runs them group by group (a grid of 8 vpx ngroups workgroups).
__device__ __forceinline__ bool radial_item(int order, int ngroups, int nvec, int& v, int& gi) {
  if (order == 0) {
    const int slot = xcd_slot(ngroups * nvec);
    v = slot / ngroups;
    gi = slot - v * ngroups;
    return slot < ngroups * nvec;
  }
  const int vpx = (nvec + 7) / 8;
  const int x = (int)(blockIdx.x & 7), i = (int)(blockIdx.x >> 3);
  gi = i / vpx;
  v = x * vpx + (i - gi * vpx);
  return gi < ngroups && v < nvec;
}

inline int radial_grid(int order, int nwg, int ngroups, int nvec) {
  return order == 0 ? nwg : 8 * ((nvec + 7) / 8) * ngroups;
}

// ------------------------------------------------------------------ radix DFTs
// In-register R-point DFT, y_p = sum_q v_q exp(s 2 pi i p q / R), s = -1
// (forward) or +1 (inverse).
template <typename T>
__device__ __forceinline__ void dft2(cplx<T>* v, T) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <typename T>
__device__ __forceinline__ void dft3(cplx<T>* v, T s) {
  const T h = (T)0.86602540378443864676;  // sqrt(3)/2
  cplx<T> t1 = cadd(v[1], v[2]);
  cplx<T> t2 = {v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
  cplx<T> d = csub(v[1], v[2]);
  cplx<T> t3 = cmuli(cplx<T>{h * d.x, h * d.y}, s);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}
template <typename T>
__device__ __forceinline__ void dft4(cplx<T>* v, T s) {
  cplx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  cplx<T> c = cadd(v[1], v[3]), d = cmuli(csub(v[1], v[3]), s);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <typename T>
__device__ __forceinline__ void dft5(cplx<T>* v, T s) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;  // cos 2pi/5, cos 4pi/5
  const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;   // sin 2pi/5, sin 4pi/5
  cplx<T> a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
  cplx<T> b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
  cplx<T> p1 = {v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
  cplx<T> p2 = {v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
  cplx<T> q1 = cmuli(cplx<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y}, s);
  cplx<T> q2 = cmuli(cplx<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y}, s);
  v[0] = cadd(v[0], cadd(a1, a2));
  v[1] = cadd(p1, q1);
  v[4] = csub(p1, q1);
  v[2] = cadd(p2, q2);
  v[3] = csub(p2, q2);
}

template <typename T, int R>
__device__ __forceinline__ void dftR(cplx<T>* v, T s) {
  if constexpr (R == 2) dft2(v, s);
  else if constexpr (R == 3) dft3(v, s);
  else if constexpr (R == 4) dft4(v, s);
  else dft5(v, s);
}

// One Stockham radix-R pass over `nlines` lines of length N held in LDS.
// Line l starts at (rows ? rows[l] : l) * line_mul and its elements are
// `stride` apart.  All loads of the pass complete (barrier) before any store,
// so the pass runs in place.  tw[t] = exp(-2 pi i t / N).  When vmul is given
// every loaded element is first multiplied by the real vmul[offset].
template <typename T, int R>
__device__ __forceinline__ void fft_pass(cplx<T>* buf, int nlines, const int32_t* rows, int line_mul,
                                         int stride, int N, int Ns, const cplx<T>* tw, T sgn,
                                         const T* __restrict__ vmul) {
  constexpr int BMAX = (MAXGRID / R + NT - 1) / NT;
  const int NR = N / R;
  const int nb = nlines * NR;
  const int tstep = N / (Ns * R);
  cplx<T> v[BMAX][R];
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = threadIdx.x + i * NT;
    if (b < nb) {
      const int line = b / NR, j = b - line * NR;
      const int base = (rows ? rows[line] : line) * line_mul;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int off = base + (j + q * NR) * stride;
        cplx<T> x = buf[off];
        if (vmul) {
          const T s = vmul[off];
          x.x *= s;
          x.y *= s;
        }
        v[i][q] = x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = threadIdx.x + i * NT;
    if (b < nb) {
      const int line = b / NR, j = b - line * NR;
      const int base = (rows ? rows[line] : line) * line_mul;
      const int k = j % Ns;
#pragma unroll
      for (int q = 1; q < R; ++q) {
        cplx<T> w = tw[q * k * tstep];
        w.y = sgn < 0 ? w.y : -w.y;
        v[i][q] = cmul(v[i][q], w);
      }
      dftR<T, R>(v[i], sgn);
      const int o = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[base + (o + q * Ns) * stride] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename T>
__device__ void fft_lines(cplx<T>* buf, int nlines, const int32_t* rows, int line_mul, int stride,
                          const FftPlan& plan, const cplx<T>* tw, T sgn, const T* vmul) {
  int Ns = 1;
  for (int s = 0; s < plan.nf; ++s) {
    const int R = plan.f[s];
    const T* vm = (s == 0) ? vmul : nullptr;
    switch (R) {
      case 2: fft_pass<T, 2>(buf, nlines, rows, line_mul, stride, plan.n, Ns, tw, sgn, vm); break;
      case 3: fft_pass<T, 3>(buf, nlines, rows, line_mul, stride, plan.n, Ns, tw, sgn, vm); break;
      case 4: fft_pass<T, 4>(buf, nlines, rows, line_mul, stride, plan.n, Ns, tw, sgn, vm); break;
      default: fft_pass<T, 5>(buf, nlines, rows, line_mul, stride, plan.n, Ns, tw, sgn, vm); break;
    }
    Ns *= R;
  }
}

}  // namespace helic
