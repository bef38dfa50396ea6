// Device side of the helical-wave Hamiltonian library: table upload, the
// three kernels of H*X (see kernels.hpp), the transforms on their own, the
// Teter-Payne-Allan preconditioner and their C ABI entry points.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device_state.hpp"
#include "helic_internal.h"
#include "kernels.hpp"
#include "angular_fast.hpp"
#include "angular_grid.hpp"
#include "angular_split.hpp"
#include "angular_pipe.hpp"

// Stage launch; with timing events they ride on the kernel's own dispatch
// packet (start and end timestamps of that kernel, no marker packets between
// the stages).
#define HELIC_LAUNCH(K, G, B, LDS, ST, E0, E1, ...)                                  \
  do {                                                                             \
    if (E0) hipExtLaunchKernelGGL(K, G, B, LDS, ST, E0, E1, 0, __VA_ARGS__);       \
    else hipLaunchKernelGGL(K, G, B, LDS, ST, __VA_ARGS__);                         \
  } while (0)

namespace helic {

// ============================================================ kernels
// Radial inverse stage: one |n| group x one vector per workgroup.  The
// group's coefficients are staged in LDS as [k][2 * modes] (real columns),
// each wave takes 16-radius tiles.  KS bounds the k steps (of 4) of the
// widest group; up to 16 steps the table fragments of the wave's next tile
// are fetched into registers while the current tile's MFMAs run (beyond, the
// doubled registers cost more occupancy than the prefetch gains).  Groups of
// more than 12 k steps run the contraction in chunks of INV_CH steps (see the
// kernel).
constexpr int INV_CH = 2;

// Value of lane l ^ 1 (DPP quad permutation 1, 0, 3, 2; all lanes active).
__device__ __forceinline__ double swap_lane_pairs(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swap_lane_pairs(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// Largest K among modes 8 c .. 8 c + 7 of a group (one 16-column MFMA tile),
// for lane c < 64: output tiles beyond it are empty and contraction steps
// beyond it multiply zeros.  The basis stores a group's modes by K
// descending, so it is the K of the tile's first mode.
__device__ __forceinline__ int tile_kmax(const DMode* gm, int nmodes, int lane) {
  return 8 * lane < nmodes ? gm[8 * lane].K : 0;
}

// Column swizzle of the inverse kernel's coefficient block: row k stores
// column pair c at pair c ^ ((k / 2 in FP64, k / 4 in FP32) mod 8), inside
// its 16-column tile.  Rows are hs apart, an odd multiple of 16 elements, so
// without it the staging writes of consecutive k of one mode (consecutive
// threads) pile onto the same LDS banks; the MFMA B reads of a tile row stay
// a permutation of that row.
template <typename T>
__device__ __forceinline__ int inv_swz(int k) {
  return 2 * ((k >> (sizeof(T) == 8 ? 1 : 2)) & 7);
}

template <typename T, int KS>
__global__ void __launch_bounds__(NT, KS <= 12 ? 4 : 3)
k_radial_inverse(const double* __restrict__ X, int64_t ldx, T* __restrict__ GH, int nvec, int ngroups, int n_r,
                 const DGroup* __restrict__ groups, const DProb* __restrict__ probs, int order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Bs = reinterpret_cast<T*>(smem_raw);
  // work in vector-major order: the slots of one XCD run every group of a few
  // vectors, so the workgroups resident together cover adjacent rows of one
  // vector's slab (and each XCD gets an even share of the work); see radial_item
  int v, gi;
  if (!radial_item(order, ngroups, nvec, v, gi)) return;
  const DGroup gr = groups[gi];
  const DProb& pb = probs[gr.prob];
  const int nks = (gr.Kmax + 3) / 4;
  constexpr bool CHUNKED = KS > 12;
  static_assert(KS % INV_CH == 0, "chunks tile the k steps");
  const int kpad = 4 * nks;
  const int ncol = 2 * gr.nmodes;
  const int nct = (ncol + 15) / 16;
  const int hs = lds_stride(16 * nct);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nrt = (n_r + 15) / 16;
  const T* tg = reinterpret_cast<const T*>(pb.tinv) + gr.tinv_off;
  constexpr bool PF = KS <= 16;
  T anext[PF ? KS : 1];
  auto fetch = [&](int rt, T* dst) {
#pragma unroll
    for (int s = 0; s < KS; ++s)
      dst[s] = (rt < nrt && s < nks) ? tg[((int64_t)rt * nks + s) * 64 + lane] : (T)0;
  };
  if constexpr (PF) fetch(wave, anext);   // in flight while the coefficients are staged
  for (int i = threadIdx.x; i < kpad * hs; i += NT) Bs[i] = (T)0;
  __syncthreads();
  // one row (re, im) per thread and access
  const double2* xv = reinterpret_cast<const double2*>(X + col_off(pb, ldx, nvec, v) * 2) + gr.row0;
  const int32_t* row_ck = pb.row_ck;
  for (int i = threadIdx.x; i < (int)gr.nrows; i += NT) {
    const int ck = row_ck[gr.row0 + i];
    const int c = ck >> 16, k = ck & 0xffff;
    const double2 x = xv[i];
    *reinterpret_cast<typename Vec2<T>::type*>(Bs + k * hs + ((2 * c) ^ inv_swz<T>(k))) = {(T)x.x, (T)x.y};
  }
  __syncthreads();
  T* gv = GH + (slab_off(pb, nvec, n_r, v, 0) + gr.mode0) * 2;
  // k steps of column tile c: lane c holds the largest K of the tile's 8
  // modes; groups of more than 64 tiles use the group's largest K throughout
  const int ktile = tile_kmax(pb.modes + gr.mode0, gr.nmodes, lane);
  auto tile_ks = [&](int c) { return nct <= 64 ? (__builtin_amdgcn_readlane(ktile, c) + 3) / 4 : nks; };
  typedef typename Mfma<T>::acc_t acc_t;
  // lane l reads B row 4 s + l / 16, column l % 16 of each tile, at its
  // swizzled position; the XOR repeats every BP k steps
  constexpr int BP = sizeof(T) == 8 ? 4 : 8;
  const T* bcol[BP];
#pragma unroll
  for (int s = 0; s < BP; ++s) bcol[s] = Bs + (lane >> 4) * hs + ((lane & 15) ^ inv_swz<T>((lane >> 4) + 4 * s));
  for (int rt = wave; rt < nrt; rt += NT / 64) {
    T a[KS];
    if constexpr (PF) {
#pragma unroll
      for (int s = 0; s < KS; ++s) a[s] = anext[s];
      fetch(rt + NT / 64, anext);
    } else {
      fetch(rt, a);
    }
    // two column tiles at a time: independent accumulators interleave; rows
    // beyond a mode's own K are zero in Bs.  With CHUNKED (groups of more
    // than 12 k steps, where the one-step form waited on each MFMA's LDS
    // read; with at most 12 steps four workgroups share a CU and hide it, and
    // a chunk buffer would not fit their registers) the K of a pair's first
    // tile also bounds its second's (modes by K descending), so the
    // contraction runs in chunks of INV_CH steps with no test inside a chunk,
    // the next chunk's B fragments read while the current chunk's MFMAs run.
    // The extra steps add exact zeros: below the group's nks the rows beyond
    // each mode's K are zero, beyond it the table fragments are (those reads
    // stay on the last row)
    for (int ct = 0; ct < nct; ct += 2) {
      const bool two = ct + 1 < nct;
      const int ks0 = tile_ks(ct);
      acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
      if constexpr (CHUNKED) {
        const int ct1 = two ? ct + 1 : ct;     // a lone last tile reads its own columns twice
        T bn0[INV_CH], bn1[INV_CH];
        auto read_chunk = [&](int c) {
#pragma unroll
          for (int u = 0; u < INV_CH; ++u) {
            const int s = INV_CH * c + u;
            const int sr = s < nks ? s : nks - 1;
            bn0[u] = bcol[s % BP][4 * sr * hs + 16 * ct];
            bn1[u] = bcol[s % BP][4 * sr * hs + 16 * ct1];
          }
        };
        if (ks0 > 0) read_chunk(0);
#pragma unroll
        for (int c = 0; c < KS / INV_CH; ++c) {
          if (INV_CH * c >= ks0) break;
          T b0[INV_CH], b1[INV_CH];
#pragma unroll
          for (int u = 0; u < INV_CH; ++u) {
            b0[u] = bn0[u];
            b1[u] = bn1[u];
          }
          if (c + 1 < KS / INV_CH && INV_CH * (c + 1) < ks0) read_chunk(c + 1);
#pragma unroll
          for (int u = 0; u < INV_CH; ++u) {
            acc0 = Mfma<T>::op(a[INV_CH * c + u], b0[u], acc0);
            acc1 = Mfma<T>::op(a[INV_CH * c + u], b1[u], acc1);
          }
        }
      } else {
        const int ks1 = two ? tile_ks(ct + 1) : 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          if (s < ks0) acc0 = Mfma<T>::op(a[s], bcol[s % BP][4 * s * hs + 16 * ct], acc0);
          if (s < ks1) acc1 = Mfma<T>::op(a[s], bcol[s % BP][4 * s * hs + 16 * ct + 16], acc1);
        }
      }
      // lanes 2j and 2j + 1 hold re and im of one mode for the same four rows;
      // after a swap across the pair each lane stores two (re, im) pairs
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const acc_t& ac = q == 0 ? acc0 : acc1;
        T sw[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) sw[i] = swap_lane_pairs(ac[i]);
        const int col = 16 * (ct + q) + (lane & 15);
        if (col < ncol && (q == 0 || two)) {
          const bool odd = lane & 1;
          T* dst = gv + (col & ~1);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = 16 * rt + Mfma<T>::row(lane, odd ? 2 * h + 1 : 2 * h);
            const T re = odd ? sw[2 * h + 1] : ac[2 * h];
            const T im = odd ? ac[2 * h + 1] : sw[2 * h];
            if (r < n_r) *reinterpret_cast<typename Vec2<T>::type*>(dst + (int64_t)r * pb.n_modes * 2) = {re, im};
          }
        }
      }
    }
  }
}

// GHv holds slab elements E (complex T, or bfloat16 pairs with T = float).
template <typename T, int MODE, typename E = cplx<T>>
__global__ void __launch_bounds__(NT)
k_angular(void* __restrict__ GHv, const double* __restrict__ grid_in, double* __restrict__ grid_out, int nprob, int nvec,
          int n_r, const DProb* __restrict__ probs, const int32_t* __restrict__ rows1, int nrows1,
          const cplx<T>* __restrict__ tw1g, const cplx<T>* __restrict__ tw2g, FftPlan p1, FftPlan p2, T out_scale) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n1 = p1.n, n2 = p2.n, nn = n1 * n2;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw1 = buf + nn;
  cplx<T>* tw2 = tw1 + n1;
  int32_t* rws = reinterpret_cast<int32_t*>(tw2 + n2);
  const int per = nvec * n_r;
  const int slot = xcd_slot(nprob * per);
  if (slot >= nprob * per) return;
  const int pi = slot / per, rem = slot - pi * per;
  const int r = rem / nvec, v = rem - r * nvec;
  const DProb& pb = probs[pi];
  const int n_modes = pb.n_modes;
  const DMode* modes = pb.modes;
  for (int i = threadIdx.x; i < n1; i += NT) tw1[i] = tw1g[i];
  for (int i = threadIdx.x; i < n2; i += NT) tw2[i] = tw2g[i];
  for (int i = threadIdx.x; i < nrows1; i += NT) rws[i] = rows1[i];
  E* slab = reinterpret_cast<E*>(GHv) + slab_off(pb, nvec, n_r, v, r);
  if (MODE == 2) {
    const double* gi = grid_in + (int64_t)v * nn * n_r * 2;
    for (int i = threadIdx.x; i < nn; i += NT)
      buf[i] = cplx<T>{(T)gi[((int64_t)i * n_r + r) * 2], (T)gi[((int64_t)i * n_r + r) * 2 + 1]};
    __syncthreads();
  } else {
    for (int i = threadIdx.x; i < nn; i += NT) buf[i] = cplx<T>{(T)0, (T)0};
    __syncthreads();
    for (int i = threadIdx.x; i < n_modes; i += NT) buf[modes[i].boff] = eload<T>(slab + i);
    __syncthreads();
    // inverse: theta2 lines on the occupied theta1 bins, then all theta1 lines
    fft_lines<T>(buf, nrows1, rws, n2, 1, p2, tw2, (T)1, nullptr);
    fft_lines<T>(buf, n2, nullptr, 1, n2, p1, tw1, (T)1, nullptr);
  }
  if (MODE == 1) {
    double* go = grid_out + (int64_t)v * nn * n_r * 2;
    for (int i = threadIdx.x; i < nn; i += NT) {
      go[((int64_t)i * n_r + r) * 2] = (double)buf[i].x;
      go[((int64_t)i * n_r + r) * 2 + 1] = (double)buf[i].y;
    }
    return;
  }
  // forward: theta1 lines (potential fused into the first pass), then theta2
  // lines on the bins that are kept
  const T* vm = (MODE == 0) ? reinterpret_cast<const T*>(pb.Vs) + (int64_t)r * nn : nullptr;
  fft_lines<T>(buf, n2, nullptr, 1, n2, p1, tw1, (T)-1, vm);
  fft_lines<T>(buf, nrows1, rws, n2, 1, p2, tw2, (T)-1, nullptr);
  for (int i = threadIdx.x; i < n_modes; i += NT) {
    cplx<T> x = buf[modes[i].boff];
    estore(slab + i, cplx<T>{x.x * out_scale, x.y * out_scale});
  }
}

template <typename T, int TMAX>
__global__ void __launch_bounds__(NT)
k_radial_forward(const T* __restrict__ GH, const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                 int64_t ldy, int nvec, int ngroups, int n_r, const DGroup* __restrict__ groups,
                 const DProb* __restrict__ probs, int add_kinetic, int order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Hs = reinterpret_cast<T*>(smem_raw);
  int v, gi;
  if (!radial_item(order, ngroups, nvec, v, gi)) return;   // see k_radial_inverse
  const DGroup gr = groups[gi];
  const DProb& pb = probs[gr.prob];
  const int ncol = 2 * gr.nmodes;
  const int nct = (ncol + 15) / 16;
  const int colpad = 16 * nct;
  const int hs = lds_stride(colpad);
  T* As = Hs + FWD_RCHUNK * hs;     // [k tile][step][64]
  const int nkt = (gr.Kmax + 15) / 16;
  const int ntiles = nkt * nct;
  const int nrs = (n_r + 3) / 4;
  const int n_modes = pb.n_modes;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* tg = reinterpret_cast<const T*>(pb.tfwd) + gr.tfwd_off;
  const T* hv = GH + (slab_off(pb, nvec, n_r, v, 0) + gr.mode0) * 2;
  const DMode* modes = pb.modes;
  const double* kappa = pb.kappa;
  const double* xv = add_kinetic ? X + col_off(pb, ldx, nvec, v) * 2 : nullptr;
  double* yv = Y + col_off(pb, ldy, nvec, v) * 2;
  typedef typename Mfma<T>::acc_t acc_t;
  for (int tbase = 0; tbase < ntiles; tbase += (NT / 64) * TMAX) {
    acc_t acc[TMAX];
    int aoff[TMAX], boff[TMAX];   // per tile: LDS offsets of its A rows and B columns
#pragma unroll
    for (int i = 0; i < TMAX; ++i) {
      acc[i] = acc_t{0, 0, 0, 0};
      const int t = tbase + wave + (NT / 64) * i;
      const int kt = t / nct, ct = t - kt * nct;
      aoff[i] = kt * (FWD_RCHUNK / 4) * 64 + lane;
      boff[i] = (lane >> 4) * hs + 16 * ct + (lane & 15);
    }
    for (int r0 = 0; r0 < n_r; r0 += FWD_RCHUNK) {
      __syncthreads();
      for (int i = threadIdx.x; i < FWD_RCHUNK * colpad; i += NT) {
        const int rr = i / colpad, col = i - rr * colpad;
        const int r = r0 + rr;
        Hs[rr * hs + col] = (r < n_r && col < ncol) ? hv[(int64_t)r * n_modes * 2 + col] : (T)0;
      }
      // the table fragments of this chunk (all k tiles, FWD_RCHUNK / 4 steps)
      for (int i = threadIdx.x; i < nkt * (FWD_RCHUNK / 4) * 64; i += NT) {
        const int ln = i & 63, q = i >> 6;
        const int kt = q / (FWD_RCHUNK / 4), s = q - kt * (FWD_RCHUNK / 4);
        const int rs = r0 / 4 + s;
        As[i] = rs < nrs ? tg[((int64_t)kt * nrs + rs) * 64 + ln] : (T)0;
      }
      __syncthreads();
      const int steps = min(FWD_RCHUNK / 4, nrs - r0 / 4);
#pragma unroll
      for (int i = 0; i < TMAX; ++i) {
        if (tbase + wave + (NT / 64) * i < ntiles) {
#pragma unroll
          for (int s = 0; s < FWD_RCHUNK / 4; ++s)
            if (s < steps) acc[i] = Mfma<T>::op(As[aoff[i] + s * 64], Hs[boff[i] + 4 * s * hs], acc[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TMAX; ++i) {
      const int t = tbase + wave + (NT / 64) * i;
      if (t >= ntiles) continue;
      const int kt = t / nct, ct = t - kt * nct;
      const int col = 16 * ct + (lane & 15);
      const int c = col >> 1, ri = col & 1;
      if (c >= gr.nmodes) continue;
      const DMode md = modes[gr.mode0 + c];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * kt + Mfma<T>::row(lane, j);
        if (k < md.K) {
          const int64_t row = md.row0 + k;
          double y = (double)acc[i][j];
          if (add_kinetic) y += kappa[row] * xv[2 * row + ri];
          yv[2 * row + ri] = y;
        }
      }
    }
  }
}

// LDS of the pipelined forward kernel: the chunk staging (RC slab rows of
// stride hs, then kt_max x RC/4 table fragments), padded to 16 bytes, then
// the per-group mode table and kappa x rows.
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }
__host__ __device__ constexpr size_t fwd_pf_stage_bytes(int rc, int hs, int kt_max, size_t elem) {
  return align16(((size_t)rc * hs + (size_t)kt_max * (rc / 4) * 64) * elem);
}

// Radial forward stage with software pipelining: the slab rows and table
// fragments of the next FWD_PF_RC radii are fetched into registers while the
// MFMAs run on the current ones from LDS, so global-memory latency overlaps
// the contractions.  Same tiles, layout and epilogue as k_radial_forward
// with 4 register tiles per wave.  Staging: wave w moves radii
// w * RC/4 ... of each chunk, lane l column pairs 2 (l + 64 b) + {0, 1}
// (b < CB / 2), so colpad <= 64 CB; at most FWD_PF_KT k tiles per group.
// Workgroups per CU its registers are held to: FP32 with 4 tiles and 2
// staged columns fits four, other FP32 forms two (fewer spill otherwise).
template <typename T, int CB, int TM>
constexpr int fwd_pf_min_wgs() {
  return sizeof(T) == 8 ? 1 : (TM == 4 && CB == 2 ? 4 : 2);
}

template <typename T, int CB, int TM>
__global__ void __launch_bounds__(NT, (fwd_pf_min_wgs<T, CB, TM>()))
k_radial_forward_pf(const T* __restrict__ GH, const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                    int64_t ldy, int nvec, int ngroups, int n_r, const DGroup* __restrict__ groups,
                    const DProb* __restrict__ probs, int flags, int order) {
  // flags bit 0: add kappa x; bit 1: stage kappa x of the group's rows in LDS
  const bool add_kinetic = flags & 1, kx_lds = (flags & 3) == 3;
  constexpr int RC = FWD_PF_RC, RW = FWD_PF_RC / (NT / 64), KTM = FWD_PF_KT;
  constexpr int SPW = (RC / 4) / (NT / 64);   // table steps (of 4 radii) each wave stages per chunk
  static_assert(SPW >= 1 && SPW * (NT / 64) * 4 == RC, "chunk must split evenly over the waves");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Hs = reinterpret_cast<T*>(smem_raw);
  int v, gi;
  if (!radial_item(order, ngroups, nvec, v, gi)) return;   // see k_radial_inverse
  const DGroup gr = groups[gi];
  const DProb& pb = probs[gr.prob];
  const int ncol = 2 * gr.nmodes;
  const int nct = (ncol + 15) / 16;
  const int colpad = 16 * nct;
  const int hs = lds_stride(colpad);
  T* As = Hs + RC * hs;     // [k tile][step][64]
  // the group's mode table (first row relative to the group, K) and, when
  // LDS allows, kappa x of its rows, staged at the start so the epilogue
  // does not wait on global memory after the contractions
  int32_t* mtab = reinterpret_cast<int32_t*>(smem_raw + fwd_pf_stage_bytes(RC, hs, KTM, sizeof(T)));
  double* kxs = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(mtab) + align16(8 * (size_t)gr.nmodes));
  const int nkt = (gr.Kmax + 15) / 16;
  const int ntiles = nkt * nct;
  const int nrs = (n_r + 3) / 4;
  const int64_t rstride = (int64_t)pb.n_modes * 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* tg = reinterpret_cast<const T*>(pb.tfwd) + gr.tfwd_off;
  const T* hv = GH + (slab_off(pb, nvec, n_r, v, 0) + gr.mode0) * 2;
  const DMode* modes = pb.modes;
  const double* kappa = pb.kappa;
  const double* xv = add_kinetic ? X + col_off(pb, ldx, nvec, v) * 2 : nullptr;
  double* yv = Y + col_off(pb, ldy, nvec, v) * 2;
  for (int c = threadIdx.x; c < gr.nmodes; c += NT) {
    const DMode md = modes[gr.mode0 + c];
    mtab[2 * c] = (int32_t)(md.row0 - gr.row0);
    mtab[2 * c + 1] = md.K;
  }
  if (kx_lds)
    for (int i = threadIdx.x; i < 2 * gr.nrows; i += NT) kxs[i] = kappa[gr.row0 + (i >> 1)] * xv[2 * gr.row0 + i];
  typedef typename Mfma<T>::acc_t acc_t;
  const int nchunk = (n_r + RC - 1) / RC;
  const int ktile = tile_kmax(modes + gr.mode0, gr.nmodes, lane);   // see k_radial_inverse
  T hreg[RW][CB], areg[KTM][SPW];
  // lane l moves column pairs 2 (l + 64 b) + {0, 1} (re, im of one mode) as
  // one 2-element access
  typedef typename Vec2<T>::type T2;
  auto fetch = [&](int r0) {
#pragma unroll
    for (int a = 0; a < RW; ++a) {
      const int r = r0 + wave * RW + a;
      const T* src = hv + (int64_t)r * rstride;
#pragma unroll
      for (int b = 0; b < CB / 2; ++b) {
        const int col = 2 * (lane + 64 * b);
        T2 pr = {(T)0, (T)0};
        if (r < n_r && col < ncol) pr = *reinterpret_cast<const T2*>(src + col);
        hreg[a][2 * b] = pr.x;
        hreg[a][2 * b + 1] = pr.y;
      }
    }
    // table fragments: thread (wave, lane) takes steps wave * SPW + e of
    // every k tile
    const int rs0 = r0 / 4 + wave * SPW;
#pragma unroll
    for (int kt = 0; kt < KTM; ++kt)
#pragma unroll
      for (int e = 0; e < SPW; ++e)
        areg[kt][e] = (kt < nkt && rs0 + e < nrs) ? tg[((int64_t)kt * nrs + rs0 + e) * 64 + lane] : (T)0;
  };
  auto store = [&]() {
#pragma unroll
    for (int a = 0; a < RW; ++a)
#pragma unroll
      for (int b = 0; b < CB / 2; ++b) {
        const int col = 2 * (lane + 64 * b);
        if (col < colpad) *reinterpret_cast<T2*>(Hs + (wave * RW + a) * hs + col) = T2{hreg[a][2 * b], hreg[a][2 * b + 1]};
      }
#pragma unroll
    for (int kt = 0; kt < KTM; ++kt)
      if (kt < nkt) {
#pragma unroll
        for (int e = 0; e < SPW; ++e) As[(kt * (RC / 4) + wave * SPW + e) * 64 + lane] = areg[kt][e];
      }
  };
  for (int tbase = 0; tbase < ntiles; tbase += (NT / 64) * TM) {
    acc_t acc[TM];
    int aoff[TM], boff[TM];
    bool live[TM];   // the tile has rows k < K for some of its modes
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      acc[i] = acc_t{0, 0, 0, 0};
      const int t = tbase + wave + (NT / 64) * i;
      const int kt = t / nct, ct = t - kt * nct;
      aoff[i] = kt * (RC / 4) * 64 + lane;
      boff[i] = (lane >> 4) * hs + 16 * ct + (lane & 15);
      live[i] = t < ntiles && (nct > 64 || 16 * kt < __builtin_amdgcn_readlane(ktile, ct));
    }
    fetch(0);
    for (int c = 0; c < nchunk; ++c) {
      __syncthreads();
      store();
      __syncthreads();
      if (c + 1 < nchunk) fetch((c + 1) * RC);
      const int steps = min(RC / 4, nrs - c * (RC / 4));
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        if (live[i]) {
#pragma unroll
          for (int s = 0; s < RC / 4; ++s)
            if (s < steps) acc[i] = Mfma<T>::op(As[aoff[i] + s * 64], Hs[boff[i] + 4 * s * hs], acc[i]);
        }
      }
    }
    // lanes 2j and 2j + 1 hold re and im of one mode for the same rows k;
    // after a swap across the pair each lane writes two complex rows of Y
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int t = tbase + wave + (NT / 64) * i;
      if (!live[i]) continue;   // uniform over the wave
      T sw[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) sw[j] = swap_lane_pairs(acc[i][j]);
      const int kt = t / nct, ct = t - kt * nct;
      const int col = 16 * ct + (lane & 15);
      const int c = col >> 1;
      const bool odd = lane & 1;
      if (c >= gr.nmodes) continue;
      const int roff = mtab[2 * c], K = mtab[2 * c + 1];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 16 * kt + Mfma<T>::row(lane, odd ? 2 * h + 1 : 2 * h);
        if (k < K) {
          const int lr = roff + k;
          double2 y = {(double)(odd ? sw[2 * h + 1] : acc[i][2 * h]), (double)(odd ? acc[i][2 * h + 1] : sw[2 * h])};
          if (kx_lds) {
            y.x += kxs[2 * lr];
            y.y += kxs[2 * lr + 1];
          } else if (add_kinetic) {
            const double kp = kappa[gr.row0 + lr];
            const double2 x = reinterpret_cast<const double2*>(xv)[gr.row0 + lr];
            y.x += kp * x.x;
            y.y += kp * x.y;
          }
          reinterpret_cast<double2*>(yv)[gr.row0 + lr] = y;
        }
      }
    }
  }
}

}  // namespace helic
#include "radial_bf16.hpp"
namespace helic {

// Angular mean of the potential per radius: vbar[r] = sum_{i1,i2} Vs[r][i1][i2]
// (Vs carries 1 / (n_t1 n_t2)); fixed-order block reduction.
__global__ void __launch_bounds__(NT) k_angular_mean(const double* __restrict__ Vs, int nang, double* __restrict__ vbar) {
  __shared__ double red[NT];
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nang; i += NT) acc += Vs[(int64_t)r * nang + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) vbar[r] = red[0];
}

// Diagonal of the potential term per row: the angular factors of a basis
// function have unit modulus, so V_ii = sum_r (2 pi tau R^2 w_r xi(r)) xi(r)
// vbar(r) depends on (|n|, k) only; one workgroup per |n| group reads both
// packed radial tables (forward table = 2 pi tau R^2 w_r xi, inverse = xi).
__global__ void __launch_bounds__(NT)
k_potential_diagonal(const DGroup* __restrict__ groups, const int32_t* __restrict__ row_ck,
                     const double* __restrict__ tinv, const double* __restrict__ tfwd,
                     const double* __restrict__ vbar, int n_r, double* __restrict__ vdiag) {
  __shared__ double per_k[4 * KS_MAX];
  const DGroup g = groups[blockIdx.x];
  const int nks = (g.Kmax + 3) / 4, nrs = (n_r + 3) / 4;
  for (int k = threadIdx.x; k < g.Kmax; k += NT) {
    double acc = 0.0;
    for (int l = 0; l < n_r; ++l) {
      const double xi = tinv[g.tinv_off + ((int64_t)(l / 16) * nks + k / 4) * FRAG + (l % 16) + 16 * (k % 4)];
      const double wf = tfwd[g.tfwd_off + ((int64_t)(k / 16) * nrs + l / 4) * FRAG + (k % 16) + 16 * (l % 4)];
      acc += wf * xi * vbar[l];
    }
    per_k[k] = acc;
  }
  __syncthreads();
  for (int64_t row = g.row0 + threadIdx.x; row < g.row0 + g.nrows; row += NT) vdiag[row] = per_k[row_ck[row] & 0xffff];
}

constexpr double PI_D = 3.14159265358979323846;

// Y_v = i f .* X_v for nv columns of L complex rows (App. C: the coefficients
// of a theta derivative, f = 2 pi m or 2 pi n per row).
__global__ void __launch_bounds__(NT)
k_scale_imag(const double* __restrict__ X, int64_t ldx, double* __restrict__ Y, int64_t L, int nv,
             const double* __restrict__ f) {
  const int v = blockIdx.y;
  const double2* x = reinterpret_cast<const double2*>(X) + (int64_t)v * ldx;
  double2* y = reinterpret_cast<double2*>(Y) + (int64_t)v * L;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < L; i += (int64_t)gridDim.x * NT) {
    const double2 a = x[i];
    y[i] = double2{-f[i] * a.y, f[i] * a.x};
  }
}

// Helical to Cartesian derivatives at every grid point, in place (App. C, eq.
// Cartesian_Derivatives): G holds three blocks of nv grids (E_theta1,
// E_theta2, E_r), each grid n1 x n2 x n_r complex values with r fastest.
// phi = 2 pi (alpha theta1 + theta2); E_x = -sin(phi) E_theta2 / (2 pi r) +
// cos(phi) E_r, E_y = cos(phi) E_theta2 / (2 pi r) + sin(phi) E_r,
// E_z = (E_theta1 - alpha E_theta2) / tau.
__global__ void __launch_bounds__(NT)
k_cartesian(double* __restrict__ G, int nv, int n1, int n2, int n_r, const double* __restrict__ rg, double alpha,
            double tau, int ncyc) {
  const int64_t npts = (int64_t)n1 * n2 * n_r;
  double2* g = reinterpret_cast<double2*>(G);
  const int v = blockIdx.y;
  for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < npts; p += (int64_t)gridDim.x * NT) {
    const int l = (int)(p % n_r);
    const int64_t a = p / n_r;
    const int i2 = (int)(a % n2), i1 = (int)(a / n2);
    const double phi = 2.0 * PI_D * (alpha * ((double)i1 / n1) + (double)i2 / ((double)ncyc * n2));
    double sn, cs;
    sincos(phi, &sn, &cs);
    const double ir = 1.0 / (2.0 * PI_D * rg[l]);
    double2* e1 = g + (int64_t)v * npts + p;
    double2* e2 = g + ((int64_t)nv + v) * npts + p;
    double2* er = g + (2 * (int64_t)nv + v) * npts + p;
    const double2 t1 = *e1, t2 = *e2, tr = *er;
    *e1 = double2{-sn * ir * t2.x + cs * tr.x, -sn * ir * t2.y + cs * tr.y};
    *e2 = double2{cs * ir * t2.x + sn * tr.x, cs * ir * t2.y + sn * tr.y};
    *er = double2{(t1.x - alpha * t2.x) / tau, (t1.y - alpha * t2.y) / tau};
  }
}

// Electron density (Sec. 4.2): rho[p] (+)= sum_v occ[v] |g_v[p]|^2 over the
// npts grid points, g holding nv real-space grids of complex values.  One
// thread per point, states in order, so the sum is deterministic.  HBM-bound:
// 16 bytes read per state and point.
__global__ void __launch_bounds__(NT)
k_density_accum(const double* __restrict__ g, int nv, int64_t npts, const double* __restrict__ occ,
                double* __restrict__ rho, int accumulate) {
  const double2* z = reinterpret_cast<const double2*>(g);
  for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < npts; p += (int64_t)gridDim.x * NT) {
    double s = accumulate ? rho[p] : 0.0;
    for (int v = 0; v < nv; ++v) {
      const double2 c = z[(int64_t)v * npts + p];
      s += occ[v] * (c.x * c.x + c.y * c.y);
    }
    rho[p] = s;
  }
}

// Vs[r][i1][i2] = scale * V[i1][i2][r] (and the single-precision copy)
__global__ void __launch_bounds__(NT)
k_relayout_potential(const double* __restrict__ V, double* __restrict__ Vs, float* __restrict__ Vsf,
                     int n1, int n2, int n_r, double scale) {
  const int64_t total = (int64_t)n1 * n2 * n_r;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
    const int64_t r = i / ((int64_t)n1 * n2), rem = i - r * n1 * n2;
    const double x = scale * V[rem * n_r + r];
    Vs[i] = x;
    Vsf[i] = (float)x;
  }
}

// Vh[r][j][d] = 1/(n1 n2) sum_i V[i][j][r] exp(-i 2 pi (d - (mpad - 1)) i / n1)
__global__ void __launch_bounds__(NT)
k_potential_spectrum(const double* __restrict__ V, double* __restrict__ Vh, float* __restrict__ Vhf, int n1,
                     int n2, int n_r, int mpad) {
  const int nd = 2 * mpad - 1;
  const int64_t total = (int64_t)n_r * n2 * nd;
  const double PI2 = 6.283185307179586477;
  for (int64_t idx = blockIdx.x * (int64_t)NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int d = (int)(idx % nd);
    const int64_t rj = idx / nd;
    const int j = (int)(rj % n2), r = (int)(rj / n2);
    const int dd = d - (mpad - 1);
    double re = 0.0, im = 0.0;
    for (int i = 0; i < n1; ++i) {
      int t = (dd * i) % n1;
      if (t < 0) t += n1;
      double sn, cs;
      sincos(PI2 * t / n1, &sn, &cs);
      const double x = V[((int64_t)i * n2 + j) * n_r + r];
      re += x * cs;
      im -= x * sn;
    }
    const double sc = 1.0 / ((double)n1 * n2);
    Vh[2 * idx] = re * sc;
    Vh[2 * idx + 1] = im * sc;
    Vhf[2 * idx] = (float)(re * sc);
    Vhf[2 * idx + 1] = (float)(im * sc);
  }
}

// Teter-Payne-Allan: partial sums of kappa |r|^2 and |r|^2 per (chunk, column)
__global__ void __launch_bounds__(NT)
k_tpa_partial(const double* __restrict__ Rr, int64_t ldr, const double* __restrict__ kappa, int64_t L,
              int nchunk, double* __restrict__ part) {
  __shared__ double s_num[NT], s_den[NT];
  const int c = blockIdx.x, j = blockIdx.y;
  const int64_t per = (L + nchunk - 1) / nchunk;
  const int64_t lo = c * per, hi = std::min(L, lo + per);
  double num = 0.0, den = 0.0;
  const double* rc = Rr + (int64_t)j * ldr * 2;
  for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
    const double a = rc[2 * i], b = rc[2 * i + 1];
    const double m2 = a * a + b * b;
    den += m2;
    num += kappa[i] * m2;
  }
  s_num[threadIdx.x] = num;
  s_den[threadIdx.x] = den;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_num[threadIdx.x] += s_num[threadIdx.x + s];
      s_den[threadIdx.x] += s_den[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)j * nchunk + c) * 2] = s_num[0];
    part[((int64_t)j * nchunk + c) * 2 + 1] = s_den[0];
  }
}

__global__ void __launch_bounds__(NT)
k_tpa_apply(const double* __restrict__ Rr, int64_t ldr, double* __restrict__ W, int64_t ldw,
            const double* __restrict__ kappa, int64_t L, int nchunk, const double* __restrict__ part) {
  const int j = blockIdx.y;
  double num = 0.0, den = 0.0;
  for (int c = 0; c < nchunk; ++c) {   // fixed order: deterministic
    num += part[((int64_t)j * nchunk + c) * 2];
    den += part[((int64_t)j * nchunk + c) * 2 + 1];
  }
  const double T = den > 0.0 ? num / den : 0.0;
  const double* rc = Rr + (int64_t)j * ldr * 2;
  double* wc = W + (int64_t)j * ldw * 2;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < L; i += (int64_t)gridDim.x * NT) {
    double f = 0.0;
    if (T > 0.0) {
      const double g = kappa[i] / T;
      const double num3 = 27.0 + g * (18.0 + g * (12.0 + 8.0 * g));
      f = num3 / (num3 + 16.0 * g * g * g * g);
    }
    wc[2 * i] = f * rc[2 * i];
    wc[2 * i + 1] = f * rc[2 * i + 1];
  }
}

// ============================================================ host side
#define HIP_TRY(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(HELIC_ERR_HIP, std::string(#call) + " (line " + std::to_string(__LINE__) + "): " + \
                                     hipGetErrorString(e_));                            \
  } while (0)

namespace {

template <typename T>
helic_status upload(const std::vector<T>& host, T** dptr) {
  if (host.empty()) {
    *dptr = nullptr;
    return HELIC_OK;
  }
  HIP_TRY(hipMalloc((void**)dptr, sizeof(T) * host.size()));
  HIP_TRY(hipMemcpy(*dptr, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
  return HELIC_OK;
}

// Output tiles of the widest group (16 k x 16 columns each); the radial
// forward kernel keeps 4 * TMAX of them in registers per pass over r.
int fwd_tiles_max(const helic_basis_s* h) {
  int t = 0;
  for (const Group& g : h->groups) t = std::max(t, ((g.Kmax + 15) / 16) * ((2 * g.nmodes + 15) / 16));
  return t;
}

// Register tiles per wave: 4 by default.  Measured on MI355X, covering the
// widest group in one pass (8-16 tiles) costs more in occupancy than the
// extra passes over the LDS-staged slab.  HELIC_FWD_TMAX = 8, 12 or 16
// selects a larger variant (for comparison).
int fwd_tmax_for(int tiles) {
  (void)tiles;
  if (const char* e = std::getenv("HELIC_FWD_TMAX")) {
    const int v = std::atoi(e);
    if (v == 4 || v == 8 || v == 12 || v == 16) return v;
  }
  return 4;
}

// The pipelined radial forward kernel (variant 0) when the basis fits its
// register staging; HELIC_FWD_PF=0 keeps the plain one.
size_t fwd_pf_lds_bytes(const helic_basis_s* h, size_t elem, bool kx_lds) {
  size_t tail = 0;   // mode table (and kappa x rows) of the largest group
  for (const Group& g : h->groups)
    tail = std::max(tail, align16(8 * (size_t)g.nmodes) + (kx_lds ? 16 * (size_t)g.nrows : 0));
  return fwd_pf_stage_bytes(FWD_PF_RC, lds_stride(h->max_colpad), FWD_PF_KT, elem) + tail;
}

// kappa x is staged in LDS when that still leaves room for the workgroups
// per CU the kernel's registers allow (two in FP64, three in FP32).
bool fwd_pf_kx_lds(const helic_basis_s* h, size_t elem) {
  return fwd_pf_lds_bytes(h, elem, true) <= (size_t)160 * 1024 / (elem == 8 ? 2 : 3);
}

bool fwd_pf_ok(const helic_basis_s* h) {
  if (const char* e = std::getenv("HELIC_FWD_PF"))
    if (e[0] == '0') return false;
  return h->max_colpad <= FWD_PF_COLS && (h->max_kpad + 15) / 16 <= FWD_PF_KT &&
         fwd_pf_lds_bytes(h, sizeof(double), false) <= 160 * 1024;
}


// Register k steps of the inverse kernel: the smallest of 8, 12, 16, 24 that
// covers the widest group (up to 12 the kernel fits four workgroups per CU).
int inv_ks_for(const helic_basis_s* h) {
  const int nks = h->max_kpad / 4;
  return nks <= 8 ? 8 : nks <= 12 ? 12 : nks <= 16 ? 16 : 24;
}

template <typename T>
void launch_radial_inverse(int ks, int nwg, size_t lds, hipStream_t st, const double* X, int64_t ldx, T* gh,
                           int nvec, int ngroups, int n_r, const DGroup* groups, const DProb* probs, int order,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  nwg = radial_grid(order, nwg, ngroups, nvec);
  if (ks <= 8)
    HELIC_LAUNCH((k_radial_inverse<T, 8>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r, groups,
                       probs, order);
  else if (ks <= 12)
    HELIC_LAUNCH((k_radial_inverse<T, 12>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r,
                       groups, probs, order);
  else if (ks <= 16)
    HELIC_LAUNCH((k_radial_inverse<T, 16>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r,
                       groups, probs, order);
  else
    HELIC_LAUNCH((k_radial_inverse<T, 24>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r,
                       groups, probs, order);
}

// Register tiles per wave of the pipelined radial forward kernel: 8 in FP64
// (one pass over the slab for groups of up to 32 tiles); in FP32 4 (four
// workgroups per CU) unless the widest group then needs a second pass over
// the slab (more than 16 tiles).  Measured best on the nanotube and nanowire
// workloads; HELIC_FWD_PF_TILES = 4 or 8 overrides.
int fwd_pf_tiles(bool fp64, int tiles_max) {
  const char* e = std::getenv("HELIC_FWD_PF_TILES");
  if (e && (e[0] == '4' || e[0] == '8' || (fp64 && e[0] == '9'))) return e[0] - '0';
  // FP64 groups of 33 to 36 tiles (the nanowire's widest): 9 tiles per wave
  // keep them to one pass over the slab
  if (fp64 && tiles_max > 8 * (NT / 64) && tiles_max <= 9 * (NT / 64)) return 9;
  return fp64 || tiles_max > 4 * (NT / 64) ? 8 : 4;
}

// One launch of the radial forward stage with the smallest register tile
// count that covers every group in one pass.
template <typename T>
void launch_radial_forward(int tmax, int nwg, size_t lds, hipStream_t st, const T* gh, const double* X, int64_t ldx,
                           double* Y, int64_t ldy, int nvec, int ngroups, int n_r, const DGroup* groups,
                           const DProb* probs, int mode, int order, int tm = 8, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr) {
  nwg = radial_grid(order, nwg, ngroups, nvec);
  switch (tmax) {
    case 0:   // pipelined variants (columns staged per lane: 2 or 4 of 64; register tiles per wave)
      if constexpr (sizeof(T) == 8) {
        if (tm == 9) {
          HELIC_LAUNCH((k_radial_forward_pf<T, 2, 9>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                             ngroups, n_r, groups, probs, mode, order);
          break;
        }
      }
      if (tm == 8)
        HELIC_LAUNCH((k_radial_forward_pf<T, 2, 8>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                           ngroups, n_r, groups, probs, mode, order);
      else
        HELIC_LAUNCH((k_radial_forward_pf<T, 2, 4>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                           ngroups, n_r, groups, probs, mode, order);
      break;
    case -1:
      if (tm == 8)
        HELIC_LAUNCH((k_radial_forward_pf<T, 4, 8>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                           ngroups, n_r, groups, probs, mode, order);
      else
        HELIC_LAUNCH((k_radial_forward_pf<T, 4, 4>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                           ngroups, n_r, groups, probs, mode, order);
      break;
    case 4:
      HELIC_LAUNCH((k_radial_forward<T, 4>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec, ngroups,
                         n_r, groups, probs, mode, order);
      break;
    case 8:
      HELIC_LAUNCH((k_radial_forward<T, 8>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec, ngroups,
                         n_r, groups, probs, mode, order);
      break;
    case 12:
      HELIC_LAUNCH((k_radial_forward<T, 12>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                         ngroups, n_r, groups, probs, mode, order);
      break;
    default:
      HELIC_LAUNCH((k_radial_forward<T, 16>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec,
                         ngroups, n_r, groups, probs, mode, order);
      break;
  }
}

size_t fwd_lds_bytes(const helic_basis_s* h, size_t elem) {
  const int nkt_max = (h->max_kpad + 15) / 16;
  return ((size_t)FWD_RCHUNK * lds_stride(h->max_colpad) + (size_t)nkt_max * (FWD_RCHUNK / 4) * 64) * elem;
}

size_t angular_lds_bytes(const helic_basis_s* h, size_t elem) {
  return (size_t)h->n_t1 * h->n_t2 * 2 * elem + (size_t)(h->n_t1 + h->n_t2) * 2 * elem +
         (size_t)h->rows1.size() * sizeof(int32_t);
}

// Problem tables of a launch in its precision: FP64, FP32, or BF16 (BF16
// radial tables, FP32 potential and twiddles).
template <typename T, typename E>
const DProb* launch_probs(const LaunchSet& ls) {
  if constexpr (std::is_same<E, bf16x2>::value) return ls.probs16;
  else return std::is_same<T, double>::value ? ls.probs64 : ls.probs32;
}

// Instantiated (n_t2, padded m count, block size) of the specialised angular kernel.
struct FastVariant { int n2, mpad, ntf; };
constexpr FastVariant FAST_VARIANTS[] = {{16, 12, 256}, {16, 16, 256}, {64, 24, 256}, {64, 28, 256},
                                         {64, 32, 256}, {81, 25, 512}, {81, 32, 512}};

template <typename T>
size_t fast_lds_bytes(int n2, int mpad) {
  return ((size_t)2 * mpad * ang_rs(n2) + n2) * sizeof(cplx<T>);
}

// Tuning knobs (environment, read once per handle): vectors per angular
// workgroup and vectors per launch of the three stages.
int env_int(const char* name, int dflt, int lo, int hi) {
  const char* e = std::getenv(name);
  if (!e || !*e) return dflt;
  return std::max(lo, std::min(hi, std::atoi(e)));
}

template <typename T, typename E, int N2, int MPAD, int NTF>
helic_status set_fast_limit() {
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular_fast<T, E, N2, MPAD, NTF>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  return HELIC_OK;
}

// FP64 blocks listed here take the wave-specialised k_angular_pipe instead
// of k_angular_fast (HELIC_ANGULAR_PIPE=0 keeps k_angular_fast).  Measured
// per 64-vector block: 32 x 81 with 25 rows 0.297 against 0.367 ms, 48 x 64
// with 28 rows 0.198 against 0.242 ms, with 24 rows 0.130 against 0.135 ms
// (the last within the run-to-run spread of the box).
#define HELIC_PIPE_FOREACH(X) X(81, 25) X(64, 24) X(64, 28)
bool pipe_for(int n2, int mpad) {
  const char* e = std::getenv("HELIC_ANGULAR_PIPE");
  if (e && e[0] == '0') return false;
#define HELIC_PIPE_HAS(N2_, MP_) if (n2 == N2_ && mpad == MP_) return true;
  HELIC_PIPE_FOREACH(HELIC_PIPE_HAS)
#undef HELIC_PIPE_HAS
  return false;
}

template <typename T>
size_t pipe_lds_bytes(int n2, int mpad) {
  return ((size_t)4 * mpad * ang_rs(n2) + n2) * sizeof(cplx<T>);
}

template <typename T, typename E>
helic_status set_fast_limits() {
  if constexpr (std::is_same<T, double>::value && std::is_same<E, cplx<double>>::value) {
#define HELIC_PIPE_ATTR(N2_, MP_)                                                                     \
    HIP_TRY(hipFuncSetAttribute((const void*)k_angular_pipe<double, cplx<double>, N2_, MP_, 512>,     \
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    HELIC_PIPE_FOREACH(HELIC_PIPE_ATTR)
#undef HELIC_PIPE_ATTR
  }
  helic_status s;
  if ((s = set_fast_limit<T, E, 16, 12, 256>()) || (s = set_fast_limit<T, E, 16, 16, 256>()) ||
      (s = set_fast_limit<T, E, 64, 24, 256>()) || (s = set_fast_limit<T, E, 64, 28, 256>()) ||
      (s = set_fast_limit<T, E, 64, 32, 256>()) || (s = set_fast_limit<T, E, 81, 25, 512>()) ||
      (s = set_fast_limit<T, E, 81, 32, 512>()))
    return s;
  return HELIC_OK;
}

// Resident workgroups of the chosen angular kernel on the whole device.
template <typename T, typename E>
int fast_slots(int n2, int mpad, int ntf, int ncu, bool pipe = false) {
  int nb = 0;
  if constexpr (std::is_same<T, double>::value && std::is_same<E, cplx<double>>::value) {
    if (pipe) {
#define HELIC_PIPE_OCC(N2_, MP_)                                                                      \
      if (n2 == N2_ && mpad == MP_)                                                                   \
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_angular_pipe<double, cplx<double>, N2_, MP_, 512>, \
                                                           512, pipe_lds_bytes<double>(n2, mpad));
      HELIC_PIPE_FOREACH(HELIC_PIPE_OCC)
#undef HELIC_PIPE_OCC
      return std::max(1, nb) * std::max(1, ncu);
    }
  }
  const size_t lds = fast_lds_bytes<T>(n2, mpad);
#define HELIC_OCC_CASE(N2_, MP_, NTF_)                                                                 \
  if (n2 == N2_ && mpad == MP_ && ntf == NTF_)                                                        \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_angular_fast<T, E, N2_, MP_, NTF_>, NTF_, lds);
  HELIC_OCC_CASE(16, 12, 256)
  HELIC_OCC_CASE(16, 16, 256)
  HELIC_OCC_CASE(64, 24, 256)
  HELIC_OCC_CASE(64, 28, 256)
  HELIC_OCC_CASE(64, 32, 256)
  HELIC_OCC_CASE(81, 25, 512)
  HELIC_OCC_CASE(81, 32, 512)
#undef HELIC_OCC_CASE
  return std::max(1, nb) * std::max(1, ncu);
}

// Work split of the specialised angular kernels: ls.vchunk items per
// workgroup if set, else the fewest items per workgroup that let every
// workgroup be resident at once (one wave of workgroups, no tail).
template <typename T, typename E>
int angular_items_per_wg(const LaunchSet& ls, int nvec) {
  if (ls.vchunk > 0) return ls.vchunk;
  const int64_t total = (int64_t)ls.nprob * ls.n_r * nvec;
  const int64_t slots = std::max(1, std::is_same<E, bf16x2>::value   ? ls.ang_slots16
                                    : std::is_same<T, double>::value ? ls.ang_slots64
                                                                     : ls.ang_slots32);
  return (int)std::max<int64_t>(1, (total + slots - 1) / slots);
}

inline unsigned angular_grid_size(const LaunchSet& ls, int nvec, int ipw) {
  const int64_t total = (int64_t)ls.nprob * ls.n_r * nvec;
  const int64_t nwg = (total + ipw - 1) / ipw;
  return (unsigned)(8 * ((nwg + 7) / 8));
}

template <typename T, typename E>
helic_status launch_fast(const LaunchSet& ls, E* gh, int nvec, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr) {
  const DProb* probs = launch_probs<T, E>(ls);
  const cplx<T>* tw2 = (const cplx<T>*)(std::is_same<T, double>::value ? ls.tw2_64 : ls.tw2_32);
  const int ipw = angular_items_per_wg<T, E>(ls, nvec);
  const dim3 grid(angular_grid_size(ls, nvec, ipw));
  if constexpr (std::is_same<T, double>::value && std::is_same<E, cplx<double>>::value) {
    if (ls.pipe64) {
#define HELIC_PIPE_CASE(N2_, MP_)                                                                     \
      if (ls.n_t2 == N2_ && ls.fast_mpad == MP_) {                                                    \
        HELIC_LAUNCH((k_angular_pipe<double, cplx<double>, N2_, MP_, 512>), grid, dim3(512),            \
                     pipe_lds_bytes<double>(N2_, MP_), st, e0, e1, gh, ls.nprob, nvec, ls.n_r, probs, tw2, ipw); \
        HIP_TRY(hipGetLastError());                                                                   \
        return HELIC_OK;                                                                              \
      }
      HELIC_PIPE_FOREACH(HELIC_PIPE_CASE)
#undef HELIC_PIPE_CASE
      return fail(HELIC_ERR_STATE, "no pipelined angular kernel for this grid");
    }
  }
  const size_t lds = fast_lds_bytes<T>(ls.n_t2, ls.fast_mpad);
#define HELIC_FAST_CASE(N2_, MP_, NTF_)                                                                   \
  if (ls.n_t2 == N2_ && ls.fast_mpad == MP_ && ls.fast_ntf == NTF_) {                                    \
    HELIC_LAUNCH((k_angular_fast<T, E, N2_, MP_, NTF_>), grid, dim3(NTF_), lds, st, e0, e1, gh, ls.nprob, nvec, \
                 ls.n_r, probs, tw2, ipw);                                                              \
    HIP_TRY(hipGetLastError());                                                                         \
    return HELIC_OK;                                                                                    \
  }
  HELIC_FAST_CASE(16, 12, 256)
  HELIC_FAST_CASE(16, 16, 256)
  HELIC_FAST_CASE(64, 24, 256)
  HELIC_FAST_CASE(64, 28, 256)
  HELIC_FAST_CASE(64, 32, 256)
  HELIC_FAST_CASE(81, 25, 512)
  HELIC_FAST_CASE(81, 32, 512)
#undef HELIC_FAST_CASE
  return fail(HELIC_ERR_STATE, "no specialised angular kernel for this grid");
}

// Grids served by the split theta1 FFT kernel in FP32 arithmetic (FP32 and
// BF16 modes; theta1 size, theta2 size, padded m count, block size): the m
// range covers most of a small theta1 grid, where the column DFTs cost fewer
// operations than the M^2 convolution.  Measured against the convolution
// kernel: 32 x 81 (25 rows) FP32 0.200 vs 0.221 ms, BF16 0.221 vs 0.227 ms;
// 48 x 64 (28 rows) FP32 0.122 vs 0.136 ms, BF16 0.124 vs 0.146 ms per
// 64-vector block.  With 24 rows on 48 x 64, and in FP64 everywhere (where
// the kernel needs more registers than three waves per SIMD allow and its
// LDS exchanges are exposed), the convolution kernel measured faster.
struct SplitVariant { int n1, n2, mpad, ntf; };
constexpr SplitVariant SPLIT_VARIANTS[] = {{32, 81, 25, 384}, {48, 64, 28, 256}};
#define HELIC_SPLIT_FOREACH(X) X(32, 81, 25, 384) X(48, 64, 28, 256)

template <typename T>
size_t split_lds_bytes(int n1, int n2) {
  return ((size_t)n1 * ang_rs(n2) + n2 + n1) * sizeof(cplx<T>);
}

bool split_disabled() {
  const char* e = std::getenv("HELIC_ANGULAR_SPLIT");
  return e && e[0] == '0';
}

template <typename E>
helic_status set_split_limits() {
#define HELIC_SPLIT_ATTR(N1_, N2_, MP_, NTF_)                                                            \
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular_split<float, E, N1_, N2_, MP_, NTF_>,             \
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HELIC_SPLIT_FOREACH(HELIC_SPLIT_ATTR)
#undef HELIC_SPLIT_ATTR
  return HELIC_OK;
}

template <typename E>
int split_slots(int n1, int n2, int mpad, int ntf, int ncu) {
  int nb = 0;
  const size_t lds = split_lds_bytes<float>(n1, n2);
#define HELIC_OCC_CASE(N1_, N2_, MP_, NTF_)                                                            \
  if (n1 == N1_ && n2 == N2_ && mpad == MP_ && ntf == NTF_)                                           \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_angular_split<float, E, N1_, N2_, MP_, NTF_>, NTF_, lds);
  HELIC_SPLIT_FOREACH(HELIC_OCC_CASE)
#undef HELIC_OCC_CASE
  return std::max(1, nb) * std::max(1, ncu);
}

template <typename E>
helic_status launch_split(const LaunchSet& ls, E* gh, int nvec, hipStream_t st, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr) {
  const DProb* probs = launch_probs<float, E>(ls);
  const cplx<float>* tw2 = (const cplx<float>*)ls.tw2_32;
  const cplx<float>* tw1 = (const cplx<float>*)ls.tw1_32;
  const int ipw = angular_items_per_wg<float, E>(ls, nvec);
  const dim3 grid(angular_grid_size(ls, nvec, ipw));
  const size_t lds = split_lds_bytes<float>(ls.n_t1, ls.n_t2);
#define HELIC_SPLIT_CASE(N1_, N2_, MP_, NTF_)                                                             \
  if (ls.n_t1 == N1_ && ls.n_t2 == N2_ && ls.fast_mpad == MP_ && ls.split_ntf == NTF_) {                 \
    HELIC_LAUNCH((k_angular_split<float, E, N1_, N2_, MP_, NTF_>), grid, dim3(NTF_), lds, st, e0, e1, gh,  \
                 ls.nprob, nvec, ls.n_r, probs, tw2, tw1, ipw);                                         \
    HIP_TRY(hipGetLastError());                                                                         \
    return HELIC_OK;                                                                                    \
  }
  HELIC_SPLIT_FOREACH(HELIC_SPLIT_CASE)
#undef HELIC_SPLIT_CASE
  return fail(HELIC_ERR_STATE, "no split angular kernel for this grid");
}

// Grids served by the register-FFT angular kernel (theta1 size, theta2 size
// and its four-step factors): the automatic grids of the batched workload.
// Where the convolution kernel also applies (48 x 64, 32 x 81) it measured
// faster (the m range there is half of theta1 or the column DFT would not
// fit the registers), so it keeps precedence.
struct GridVariant {
  int n1, n2, pa, pb;
};
constexpr GridVariant GRID_VARIANTS[] = {{20, 96, 8, 12},  {20, 120, 8, 15}, {24, 120, 8, 15},
                                         {24, 135, 9, 15}, {27, 144, 12, 12}, {27, 180, 12, 15}};
constexpr int GRID_NTF = 256;

template <typename T>
size_t grid_lds_bytes(int n1, int n2) {
  return ((size_t)n1 * grid_rs(n2) + n2) * sizeof(cplx<T>);
}

template <typename T, typename E>
helic_status set_grid_limits() {
#define HELIC_GRID_ATTR(N1_, N2_, PA_, PB_)                                                              \
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular_grid<T, E, N1_, N2_, PA_, PB_, GRID_NTF>,         \
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HELIC_GRID_ATTR(20, 96, 8, 12)
  HELIC_GRID_ATTR(20, 120, 8, 15)
  HELIC_GRID_ATTR(24, 120, 8, 15)
  HELIC_GRID_ATTR(24, 135, 9, 15)
  HELIC_GRID_ATTR(27, 144, 12, 12)
  HELIC_GRID_ATTR(27, 180, 12, 15)
#undef HELIC_GRID_ATTR
  return HELIC_OK;
}

template <typename T, typename E>
int grid_slots(int n1, int n2, int ncu) {
  int nb = 0;
  const size_t lds = grid_lds_bytes<T>(n1, n2);
#define HELIC_OCC_CASE(N1_, N2_, PA_, PB_)                                                             \
  if (n1 == N1_ && n2 == N2_)                                                                         \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_angular_grid<T, E, N1_, N2_, PA_, PB_, GRID_NTF>, \
                                                       GRID_NTF, lds);
  HELIC_OCC_CASE(20, 96, 8, 12)
  HELIC_OCC_CASE(20, 120, 8, 15)
  HELIC_OCC_CASE(24, 120, 8, 15)
  HELIC_OCC_CASE(24, 135, 9, 15)
  HELIC_OCC_CASE(27, 144, 12, 12)
  HELIC_OCC_CASE(27, 180, 12, 15)
#undef HELIC_OCC_CASE
  return std::max(1, nb) * std::max(1, ncu);
}

template <typename T, typename E>
helic_status launch_grid(const LaunchSet& ls, E* gh, int nvec, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr) {
  const DProb* probs = launch_probs<T, E>(ls);
  const cplx<T>* tw2 = (const cplx<T>*)(std::is_same<T, double>::value ? ls.tw2_64 : ls.tw2_32);
  const int ipw = angular_items_per_wg<T, E>(ls, nvec);
  const dim3 grid(angular_grid_size(ls, nvec, ipw));
  const size_t lds = grid_lds_bytes<T>(ls.n_t1, ls.n_t2);
#define HELIC_GRID_CASE(N1_, N2_, PA_, PB_)                                                              \
  if (ls.n_t1 == N1_ && ls.n_t2 == N2_) {                                                               \
    HELIC_LAUNCH((k_angular_grid<T, E, N1_, N2_, PA_, PB_, GRID_NTF>), grid, dim3(GRID_NTF), lds, st, e0, e1, gh, \
                 ls.nprob, nvec, ls.n_r, probs, tw2, ipw);                                              \
    HIP_TRY(hipGetLastError());                                                                         \
    return HELIC_OK;                                                                                    \
  }
  HELIC_GRID_CASE(20, 96, 8, 12)
  HELIC_GRID_CASE(20, 120, 8, 15)
  HELIC_GRID_CASE(24, 120, 8, 15)
  HELIC_GRID_CASE(24, 135, 9, 15)
  HELIC_GRID_CASE(27, 144, 12, 12)
  HELIC_GRID_CASE(27, 180, 12, 15)
#undef HELIC_GRID_CASE
  return fail(HELIC_ERR_STATE, "no register-FFT angular kernel for this grid");
}

template <typename T>
helic_status set_lds_limits() {
  const int lim = 160 * 1024;
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse<T, 12>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse<T, 24>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_pf<T, 2, 4>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_pf<T, 4, 4>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_pf<T, 2, 8>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_pf<T, 4, 8>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  if constexpr (sizeof(T) == 8)
    HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_pf<T, 2, 9>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward<T, 12>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular<T, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular<T, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  return HELIC_OK;
}

// BF16 radial kernels: k steps (of 16) of the widest group, and LDS bytes of
// the staged coefficient columns (inverse) and slab chunk (forward).
int inv_kt16_for(int max_kpad) { return (max_kpad + 15) / 16 <= 2 ? 2 : (max_kpad + 15) / 16 <= 4 ? 4 : 6; }
size_t lds_inv16_bytes(int max_kpad, int max_colpad) {
  return (size_t)max_colpad * bf16_col_stride(16 * ((max_kpad + 15) / 16)) * sizeof(uint16_t);
}
size_t lds_fwd16_bytes(int max_colpad) {
  return fwd16_table_off(max_colpad) + (size_t)FWD16_KT * (FWD16_RC / 16) * 64 * sizeof(uint64_t);
}

void launch_radial_inverse_bf16(int kt16, int nwg, size_t lds, hipStream_t st, const double* X, int64_t ldx,
                                bf16x2* gh, int nvec, int ngroups, int n_r, const DGroup* groups, const DProb* probs,
                                int order, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  nwg = radial_grid(order, nwg, ngroups, nvec);
  if (kt16 <= 2)
    HELIC_LAUNCH((k_radial_inverse_bf16<2>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r,
                 groups, probs, order);
  else if (kt16 <= 4)
    HELIC_LAUNCH((k_radial_inverse_bf16<4>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r,
                 groups, probs, order);
  else
    HELIC_LAUNCH((k_radial_inverse_bf16<6>), dim3(nwg), dim3(NT), lds, st, e0, e1, X, ldx, gh, nvec, ngroups, n_r,
                 groups, probs, order);
}

void launch_radial_forward_bf16(int tm, int nwg, size_t lds, hipStream_t st, const bf16x2* gh, const double* X,
                                int64_t ldx, double* Y, int64_t ldy, int nvec, int ngroups, int n_r,
                                const DGroup* groups, const DProb* probs, int mode, int order,
                                hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  nwg = radial_grid(order, nwg, ngroups, nvec);
  if (tm == 12)
    HELIC_LAUNCH((k_radial_forward_bf16<12>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec, ngroups,
                 n_r, groups, probs, mode, order);
  else
    HELIC_LAUNCH((k_radial_forward_bf16<8>), dim3(nwg), dim3(NT), lds, st, e0, e1, gh, X, ldx, Y, ldy, nvec, ngroups,
                 n_r, groups, probs, mode, order);
}

// Register tiles per wave of the BF16 forward kernel: 8 (three waves per
// SIMD), also where the widest group then needs a second pass over the slab
// (measured: 12 tiles, two waves per SIMD, 22 % slower on the nanowire);
// HELIC_FWD16_TILES = 12 selects the wider variant (for comparison).
int fwd16_tiles(int tiles_max) {
  (void)tiles_max;
  const char* e = std::getenv("HELIC_FWD16_TILES");
  return (e && std::atoi(e) == 12) ? 12 : 8;
}

helic_status set_bf16_limits() {
  const int lim = 160 * 1024;
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse_bf16<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse_bf16<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_inverse_bf16<6>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_bf16<8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_radial_forward_bf16<12>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  HIP_TRY(hipFuncSetAttribute((const void*)k_angular<float, 0, bf16x2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lim));
  return HELIC_OK;
}

// HELIC_GENERIC_ANGULAR=1 forces the general angular kernel (for comparison).
bool fast_disabled() {
  const char* e = std::getenv("HELIC_GENERIC_ANGULAR");
  return e && e[0] == '1';
}

FftPlan make_plan(int n, const std::vector<int32_t>& f) {
  FftPlan p;
  std::memset(&p, 0, sizeof(p));
  p.n = n;
  p.nf = (int)f.size();
  for (size_t i = 0; i < f.size() && i < 12; ++i) p.f[i] = f[i];
  return p;
}

}  // namespace

// Scratch array of helic_apply_H_noalloc: the intermediate slabs of H*X for
// callers that cannot allocate.  One copy per GPU, loaded with the code
// object and held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the device
// symbol): it uses the address hipGetSymbolAddress returns on each device,
// taken once per device at the first handle set-up there (the device is
// current then) and kept in scratch_dev.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)HELIC_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[SCRATCH_MAX_DEVICES] = {};

helic_status scratch_setup(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(HELIC_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_dev[dev]) return HELIC_OK;
  void* ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(HELIC_ERR_HIP, "no device address for the scratch array");
  scratch_dev[dev] = ptr;
  return HELIC_OK;
}

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  return (dev >= 0 && dev < SCRATCH_MAX_DEVICES) ? scratch_dev[dev] : nullptr;
}

DProb problem_entry(const helic_basis_s* h, bool fp64, int64_t Lpre, int64_t mpre);
DProb problem_entry16(const helic_basis_s* h, int64_t Lpre, int64_t mpre);

helic_status ensure_device(helic_basis_s* h) {
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (h->dev) {
    if (h->dev->device != cur)
      return fail(HELIC_ERR_STATE, "handle was set up on another device");
    return HELIC_OK;
  }
  if (h->n_t1 * h->n_t2 > MAXGRID)
    return fail(HELIC_ERR_GRID, "n_t1 * n_t2 above the angular kernel's limit of " + std::to_string(MAXGRID) +
                                    " points");
  if (h->max_kpad / 4 > KS_MAX) return fail(HELIC_ERR_GRID, "more than 96 radial functions in one |n| group");
  if (angular_lds_bytes(h, sizeof(double)) > 160 * 1024)
    return fail(HELIC_ERR_GRID, "angular slab does not fit in LDS");
  if ((size_t)h->max_kpad * lds_stride(h->max_colpad) * sizeof(double) > 160 * 1024 ||
      fwd_lds_bytes(h, sizeof(double)) > 160 * 1024)
    return fail(HELIC_ERR_GRID, "a radial tile of the widest |n| group does not fit in LDS");
  helic_status s;
  if ((s = scratch_setup(cur)) != HELIC_OK) return s;
  DeviceState* d = new DeviceState();
  d->device = cur;
  h->dev = d;
  if ((s = set_lds_limits<double>()) != HELIC_OK) return s;
  if ((s = set_lds_limits<float>()) != HELIC_OK) return s;
  if ((s = set_bf16_limits()) != HELIC_OK) return s;
  std::vector<DGroup> dg(h->groups.size());
  for (size_t i = 0; i < h->groups.size(); ++i) {
    const Group& g = h->groups[i];
    dg[i] = DGroup{g.mode0, g.nmodes, g.Kmax, /*prob*/ 0, g.row0, g.nrows, g.tinv_off, g.tfwd_off,
                   g.tinv16_off, g.tfwd16_off};
  }
  std::vector<DMode> dm(h->modes.size());
  for (size_t i = 0; i < h->modes.size(); ++i) {
    const Mode& m = h->modes[i];
    dm[i] = DMode{m.row0, m.K, m.bin1 * h->n_t2 + m.bin2};
  }
  std::vector<float> tinv32(h->tab_inv.begin(), h->tab_inv.end());
  std::vector<float> tfwd32(h->tab_fwd.begin(), h->tab_fwd.end());
  const double PI = 3.14159265358979323846;
  std::vector<cplx<double>> tw1(h->n_t1), tw2(h->n_t2);
  std::vector<cplx<float>> tw1f(h->n_t1), tw2f(h->n_t2);
  for (int t = 0; t < h->n_t1; ++t) {
    tw1[t] = {std::cos(2 * PI * t / h->n_t1), -std::sin(2 * PI * t / h->n_t1)};
    tw1f[t] = {(float)tw1[t].x, (float)tw1[t].y};
  }
  for (int t = 0; t < h->n_t2; ++t) {
    tw2[t] = {std::cos(2 * PI * t / h->n_t2), -std::sin(2 * PI * t / h->n_t2)};
    tw2f[t] = {(float)tw2[t].x, (float)tw2[t].y};
  }
  if ((s = upload(dg, &d->groups)) || (s = upload(dm, &d->modes)) || (s = upload(h->row_ck, &d->row_ck)) ||
      (s = upload(h->kappa, &d->kappa)) || (s = upload(h->rows1, &d->rows1)) ||
      (s = upload(h->tab_inv, &d->tinv64)) || (s = upload(h->tab_fwd, &d->tfwd64)) ||
      (s = upload(tinv32, &d->tinv32)) || (s = upload(tfwd32, &d->tfwd32)) ||
      (s = upload(h->tab_inv16, &d->tinv16)) || (s = upload(h->tab_fwd16, &d->tfwd16)) ||
      (s = upload(tw1, &d->tw1)) || (s = upload(tw2, &d->tw2)) || (s = upload(tw1f, &d->tw1f)) ||
      (s = upload(tw2f, &d->tw2f)))
    return s;
  // items per angular workgroup: 0 spreads a launch evenly over the
  // resident workgroups; HELIC_VCHUNK fixes it
  d->vchunk = env_int("HELIC_VCHUNK", 0, 0, 64);
  d->apply_chunk = env_int("HELIC_APPLY_CHUNK", APPLY_CHUNK, 1, APPLY_CHUNK);
  d->plan1 = make_plan(h->n_t1, h->fac1);
  d->plan2 = make_plan(h->n_t2, h->fac2);
  // specialised angular kernel: smallest instantiated padding of the m count
  int mlo = 1 << 30, mhi = -(1 << 30);
  for (const Mode& m : h->modes) { mlo = std::min(mlo, m.m); mhi = std::max(mhi, m.m); }
  d->m_min = mlo;
  d->m_count = mhi - mlo + 1;
  d->fast_mpad = 0;
  if (!fast_disabled()) {
    for (const FastVariant& fv : FAST_VARIANTS) {
      if (fv.n2 == h->n_t2 && fv.mpad >= d->m_count && fast_lds_bytes<double>(fv.n2, fv.mpad) <= 160 * 1024 &&
          (d->fast_mpad == 0 || fv.mpad < d->fast_mpad)) {
        d->fast_mpad = fv.mpad;
        d->fast_ntf = fv.ntf;
      }
    }
  }
  d->pipe64 = d->fast_mpad && pipe_for(h->n_t2, d->fast_mpad);
  d->split_ntf = 0;
  if (d->fast_mpad && !split_disabled()) {
    for (const SplitVariant& sv : SPLIT_VARIANTS)
      if (sv.n1 == h->n_t1 && sv.n2 == h->n_t2 && sv.mpad == d->fast_mpad &&
          split_lds_bytes<float>(sv.n1, sv.n2) <= 160 * 1024)
        d->split_ntf = sv.ntf;
    if (d->split_ntf && ((s = set_split_limits<cplx<float>>()) || (s = set_split_limits<bf16x2>()))) return s;
  }
  d->grid_var = false;
  if (!d->fast_mpad && !fast_disabled()) {
    for (const GridVariant& gv : GRID_VARIANTS)
      if (gv.n1 == h->n_t1 && gv.n2 == h->n_t2 && grid_lds_bytes<double>(gv.n1, gv.n2) <= 160 * 1024)
        d->grid_var = true;
    if (d->grid_var && ((s = set_grid_limits<double, cplx<double>>()) || (s = set_grid_limits<float, cplx<float>>()) ||
                        (s = set_grid_limits<float, bf16x2>())))
      return s;
  }
  int ncu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d->device));
  if (d->grid_var) {
    d->ang_slots64 = grid_slots<double, cplx<double>>(h->n_t1, h->n_t2, ncu);
    d->ang_slots32 = grid_slots<float, cplx<float>>(h->n_t1, h->n_t2, ncu);
    d->ang_slots16 = grid_slots<float, bf16x2>(h->n_t1, h->n_t2, ncu);
  }
  if (d->fast_mpad) {
    if ((s = set_fast_limits<double, cplx<double>>()) || (s = set_fast_limits<float, cplx<float>>()) ||
        (s = set_fast_limits<float, bf16x2>()))
      return s;
    d->ang_slots64 = fast_slots<double, cplx<double>>(h->n_t2, d->fast_mpad, d->fast_ntf, ncu, d->pipe64);
    if (d->split_ntf) {
      d->ang_slots32 = split_slots<cplx<float>>(h->n_t1, h->n_t2, d->fast_mpad, d->split_ntf, ncu);
      d->ang_slots16 = split_slots<bf16x2>(h->n_t1, h->n_t2, d->fast_mpad, d->split_ntf, ncu);
    } else {
      d->ang_slots32 = fast_slots<float, cplx<float>>(h->n_t2, d->fast_mpad, d->fast_ntf, ncu);
      d->ang_slots16 = fast_slots<float, bf16x2>(h->n_t2, d->fast_mpad, d->fast_ntf, ncu);
    }
    const int rs = ang_rs(h->n_t2);
    std::vector<int32_t> mp(h->modes.size());
    for (size_t i = 0; i < h->modes.size(); ++i) {
      const int mr = h->modes[i].m - mlo;
      mp[i] = mr * rs + (h->modes[i].bin2 ^ ang_swz(h->n_t2, mr));
    }
    if ((s = upload(mp, &d->mode_pos))) return s;
    std::vector<int32_t> bm((size_t)d->fast_mpad * h->n_t2, -1);
    for (size_t i = 0; i < h->modes.size(); ++i)
      bm[(size_t)(h->modes[i].m - mlo) * h->n_t2 + h->modes[i].bin2] = (int32_t)i;
    if ((s = upload(bm, &d->blk_mode))) return s;
    const size_t nvh = (size_t)h->n_r * h->n_t2 * (2 * d->fast_mpad - 1) * 2;
    HIP_TRY(hipMalloc((void**)&d->Vh, nvh * sizeof(double)));
    HIP_TRY(hipMalloc((void**)&d->Vhf, nvh * sizeof(float)));
  }
  const size_t nv = (size_t)h->n_t1 * h->n_t2 * h->n_r;
  HIP_TRY(hipMalloc((void**)&d->Vs, nv * sizeof(double)));
  HIP_TRY(hipMalloc((void**)&d->Vsf, nv * sizeof(float)));
  std::vector<DProb> p64{problem_entry(h, true, 0, 0)}, p32{problem_entry(h, false, 0, 0)},
      p16{problem_entry16(h, 0, 0)};
  if ((s = upload(p64, &d->probs64)) || (s = upload(p32, &d->probs32)) || (s = upload(p16, &d->probs16))) return s;
  return HELIC_OK;
}

// The BF16 mode's problem entry: BF16 radial tables, FP32 potential.
DProb problem_entry16(const helic_basis_s* h, int64_t Lpre, int64_t mpre) {
  DProb p = problem_entry(h, false, Lpre, mpre);
  p.tinv = h->dev->tinv16;
  p.tfwd = h->dev->tfwd16;
  return p;
}

DProb problem_entry(const helic_basis_s* h, bool fp64, int64_t Lpre, int64_t mpre) {
  const DeviceState* d = h->dev;
  DProb p;
  std::memset(&p, 0, sizeof(p));
  p.groups = d->groups;
  p.modes = d->modes;
  p.row_ck = d->row_ck;
  p.kappa = d->kappa;
  p.tinv = fp64 ? (const void*)d->tinv64 : (const void*)d->tinv32;
  p.tfwd = fp64 ? (const void*)d->tfwd64 : (const void*)d->tfwd32;
  p.Vs = fp64 ? (const void*)d->Vs : (const void*)d->Vsf;
  p.Vh = fp64 ? (const void*)d->Vh : (const void*)d->Vhf;
  p.mode_pos = d->mode_pos;
  p.blk_mode = d->blk_mode;
  p.Lpre = Lpre;
  p.L = h->L;
  p.mpre = mpre;
  p.n_modes = (int32_t)h->modes.size();
  return p;
}

LaunchSet launch_set(const helic_basis_s* h) {
  const DeviceState* d = h->dev;
  LaunchSet ls;
  ls.groups = d->groups;
  ls.ngroups = (int)h->groups.size();
  ls.probs64 = d->probs64;
  ls.probs32 = d->probs32;
  ls.probs16 = d->probs16;
  ls.nprob = 1;
  ls.n_r = h->n_r;
  ls.n_t1 = h->n_t1;
  ls.n_t2 = h->n_t2;
  ls.lds_inv64 = (size_t)h->max_kpad * lds_stride(h->max_colpad) * sizeof(double);
  ls.lds_fwd64 = fwd_lds_bytes(h, sizeof(double));
  ls.inv_ks = inv_ks_for(h);
  ls.fwd_tmax = fwd_tmax_for(fwd_tiles_max(h));
  ls.fwd_tm64 = fwd_pf_tiles(true, fwd_tiles_max(h));
  ls.fwd_tm32 = fwd_pf_tiles(false, fwd_tiles_max(h));
  ls.fwd_tmax_plain = ls.fwd_tmax;
  ls.lds_fwd_plain64 = ls.lds_fwd64;
  ls.lds_fwd32 = ls.lds_fwd64 / 2;
  if (ls.fwd_tmax == 4 && fwd_pf_ok(h)) {
    ls.fwd_tmax = h->max_colpad <= 128 ? 0 : -1;
    ls.kx_lds64 = fwd_pf_kx_lds(h, sizeof(double));
    ls.kx_lds32 = fwd_pf_kx_lds(h, sizeof(float));
    ls.lds_fwd64 = fwd_pf_lds_bytes(h, sizeof(double), ls.kx_lds64);
    ls.lds_fwd32 = fwd_pf_lds_bytes(h, sizeof(float), ls.kx_lds32);
  }
  ls.lds_ang64 = angular_lds_bytes(h, sizeof(double));
  ls.fast_mpad = d->fast_mpad;
  ls.fast_ntf = d->fast_ntf;
  ls.split_ntf = d->split_ntf;
  ls.pipe64 = d->pipe64;
  ls.rad_order = env_int("HELIC_RADIAL_ORDER", -1, -1, 1);
  ls.grid_var = d->grid_var;
  ls.vchunk = d->vchunk;
  ls.ang_slots64 = d->ang_slots64;
  ls.ang_slots32 = d->ang_slots32;
  ls.ang_slots16 = d->ang_slots16;
  ls.lds_inv16 = lds_inv16_bytes(h->max_kpad, h->max_colpad);
  ls.lds_fwd16 = lds_fwd16_bytes(h->max_colpad);
  ls.max_colpad = h->max_colpad;
  ls.fwd_tm16 = fwd16_tiles(fwd_tiles_max(h));
  ls.rows1 = d->rows1;
  ls.nrows1 = (int)h->rows1.size();
  ls.plan1 = d->plan1;
  ls.plan2 = d->plan2;
  ls.tw1_64 = d->tw1;
  ls.tw2_64 = d->tw2;
  ls.tw1_32 = d->tw1f;
  ls.tw2_32 = d->tw2f;
  ls.gh = d->gh;
  return ls;
}

helic_status ensure_workspace(helic_basis_s* h, int nvec, size_t elem) {
  DeviceState* d = h->dev;
  const size_t need = (size_t)nvec * h->n_r * h->modes.size() * 2 * elem;
  if (need > d->gh_bytes) {
    if (d->gh) HIP_TRY(hipFree(d->gh));
    d->gh = nullptr;
    d->gh_bytes = 0;
    HIP_TRY(hipMalloc(&d->gh, need));
    d->gh_bytes = need;
  }
  return HELIC_OK;
}

// Free a handle's intermediate buffer (it is re-created by the next apply).
void release_workspace(helic_basis_s* h) {
  DeviceState* d = h->dev;
  if (!d || !d->gh) return;
  (void)hipFree(d->gh);
  d->gh = nullptr;
  d->gh_bytes = 0;
}

void device_release(helic_basis_s* h) {
  DeviceState* d = h->dev;
  if (!d) return;
  void* ptrs[] = {d->groups, d->modes, d->row_ck, d->kappa, d->rows1, d->tinv64, d->tfwd64,
                  d->tinv32, d->tfwd32, d->tw1, d->tw2, d->tw1f, d->tw2f, d->Vs, d->Vsf,
                  d->gh, d->part, d->mode_pos, d->blk_mode, d->Vh, d->Vhf, d->probs64, d->probs32, d->vdiag, d->lpc_ws,
                  d->dens_ws, d->dens_occ, d->tdinv64, d->probs_dr, d->grad_fac, d->rgrid, d->grad_ws,
                  d->tinv16, d->tfwd16, d->probs16};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  release_solver_state(d);
  delete d;
  h->dev = nullptr;
}

// The three H*X stages over a launch set (one handle or a batch) for nvec
// vectors; ldx / ldy < 0 selects the concatenated batch layout.  P names the
// precision: double or float (slabs, tables and angular arithmetic in P), or
// bf16x2 (BF16 radial contractions and slabs, FP32 angular arithmetic).
template <typename P>
helic_status launch_stages(const LaunchSet& ls, const double* X, int64_t ldx, double* Y, int64_t ldy, int nvec,
                           hipStream_t st, int mode, hipEvent_t* ev) {
  constexpr bool BF = std::is_same<P, bf16x2>::value;
  typedef typename std::conditional<BF, float, P>::type T;        // angular arithmetic
  typedef typename std::conditional<BF, bf16x2, cplx<T>>::type E;  // slab element
  const bool f64 = std::is_same<T, double>::value;
  const DProb* probs = launch_probs<T, E>(ls);
  E* gh = reinterpret_cast<E*>(ls.gh);
  const size_t sc = f64 ? 1 : 2;
  const int wg_rad = 8 * ((ls.ngroups * nvec + 7) / 8);
  // ev (optional): start and end events of each of the three kernels
  auto e = [&](int k) { return ev ? ev[k] : (hipEvent_t) nullptr; };
  // radial work order (radial_item): in FP64 and BF16 each XCD runs a block
  // of vectors group by group, so a group's tables are fetched into its L2
  // once per block (nanowire FP64: radial inverse 962 -> 703 MB, forward
  // 1,253 -> 900 MB of HBM-side traffic per launch, the same time); FP32
  // keeps the vector-major slots, which measured up to 3 % faster there
  const int order = ls.rad_order >= 0 ? ls.rad_order : (std::is_same<T, float>::value && !BF) ? 0 : 1;
  if constexpr (BF) {
    if (ls.max_colpad > FWD16_COLS)
      return fail(HELIC_ERR_UNSUPPORTED, "BF16 mode takes |n| groups of at most 128 angular modes");
    launch_radial_inverse_bf16(inv_kt16_for(4 * ls.inv_ks), wg_rad, ls.lds_inv16, st, X, ldx, gh, nvec, ls.ngroups,
                               ls.n_r, ls.groups, probs, order, e(0), e(1));
  } else {
    launch_radial_inverse<T>(ls.inv_ks, wg_rad, ls.lds_inv64 / sc, st, X, ldx, reinterpret_cast<T*>(gh), nvec,
                             ls.ngroups, ls.n_r, ls.groups, probs, order, e(0), e(1));
  }
  HIP_TRY(hipGetLastError());
  bool split = false;
  if constexpr (!std::is_same<T, double>::value) split = ls.fast_mpad && ls.split_ntf;
  if (split) {
    if constexpr (!std::is_same<T, double>::value) {
      helic_status s = launch_split<E>(ls, gh, nvec, st, e(2), e(3));
      if (s != HELIC_OK) return s;
    }
  } else if (ls.fast_mpad) {
    helic_status s = launch_fast<T, E>(ls, gh, nvec, st, e(2), e(3));
    if (s != HELIC_OK) return s;
  } else if (ls.grid_var) {
    helic_status s = launch_grid<T, E>(ls, gh, nvec, st, e(2), e(3));
    if (s != HELIC_OK) return s;
  } else {
    const int wg_ang = 8 * ((ls.nprob * nvec * ls.n_r + 7) / 8);
    const cplx<T>* tw1 = (const cplx<T>*)(f64 ? ls.tw1_64 : ls.tw1_32);
    const cplx<T>* tw2 = (const cplx<T>*)(f64 ? ls.tw2_64 : ls.tw2_32);
    HELIC_LAUNCH((k_angular<T, 0, E>), dim3(wg_ang), dim3(NT), ls.lds_ang64 / sc, st, e(2), e(3), gh, nullptr,
                 nullptr, ls.nprob, nvec, ls.n_r, probs, ls.rows1, ls.nrows1, tw1, tw2, ls.plan1, ls.plan2, (T)1);
    HIP_TRY(hipGetLastError());
  }
  if constexpr (BF) {
    launch_radial_forward_bf16(ls.fwd_tm16, wg_rad, ls.lds_fwd16, st, gh, X, ldx, Y, ldy, nvec, ls.ngroups, ls.n_r,
                               ls.groups, probs, mode, order, e(4), e(5));
  } else {
    const bool kx_lds = ls.fwd_tmax <= 0 && mode && (f64 ? ls.kx_lds64 : ls.kx_lds32);
    launch_radial_forward<T>(ls.fwd_tmax, wg_rad, f64 ? ls.lds_fwd64 : ls.lds_fwd32, st, reinterpret_cast<T*>(gh),
                             X, ldx, Y, ldy, nvec, ls.ngroups, ls.n_r, ls.groups, probs, mode | (kx_lds ? 2 : 0),
                             order, f64 ? ls.fwd_tm64 : ls.fwd_tm32, e(4), e(5));
  }
  HIP_TRY(hipGetLastError());
  return HELIC_OK;
}

template helic_status launch_stages<double>(const LaunchSet&, const double*, int64_t, double*, int64_t, int,
                                            hipStream_t, int, hipEvent_t*);
template helic_status launch_stages<float>(const LaunchSet&, const double*, int64_t, double*, int64_t, int,
                                           hipStream_t, int, hipEvent_t*);
template helic_status launch_stages<bf16x2>(const LaunchSet&, const double*, int64_t, double*, int64_t, int,
                                            hipStream_t, int, hipEvent_t*);

// Bytes per complex slab element in precision prec.
size_t slab_elem_bytes(helic_prec prec) {
  return prec == HELIC_FP64 ? 16 : prec == HELIC_FP32 ? 8 : 4;
}

helic_status launch_apply(helic_basis_s* h, helic_prec prec, const double* X, int64_t ldx, double* Y, int64_t ldy,
                          int nvec, hipStream_t st, int mode, hipEvent_t* ev = nullptr) {
  const LaunchSet ls = launch_set(h);
  return prec == HELIC_FP64   ? launch_stages<double>(ls, X, ldx, Y, ldy, nvec, st, mode, ev)
         : prec == HELIC_FP32 ? launch_stages<float>(ls, X, ldx, Y, ldy, nvec, st, mode, ev)
                              : launch_stages<bf16x2>(ls, X, ldx, Y, ldy, nvec, st, mode, ev);
}

helic_status apply_H_impl(helic_basis_s* h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                          int nvec, helic_prec prec, hipStream_t st, int chunk) {
  chunk = std::max(1, std::min(chunk, h->dev->apply_chunk));
  helic_status s = ensure_workspace(h, std::min(nvec, chunk), slab_elem_bytes(prec) / 2);
  if (s != HELIC_OK) return s;
  for (int v0 = 0; v0 < nvec; v0 += chunk) {
    const int nv = std::min(chunk, nvec - v0);
    const double* Xc = X + (int64_t)v0 * ldx * 2;
    double* Yc = Y + (int64_t)v0 * ldy * 2;
    s = launch_apply(h, prec, Xc, ldx, Yc, ldy, nv, st, 1);
    if (s != HELIC_OK) return s;
  }
  return HELIC_OK;
}

// helic_apply_H with the intermediate slabs in this device's scratch array:
// as many vectors per launch as fit (at most the usual 64).  Allocates
// nothing; the handle's own buffer is neither used nor grown.
helic_status apply_H_noalloc_impl(helic_basis_s* h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                                  int nvec, helic_prec prec, hipStream_t st) {
  void* ws = scratch_ptr(h->dev->device);
  if (!ws) return fail(HELIC_ERR_STATE, "scratch array not set up on this device");
  const size_t per_vec = (size_t)h->n_r * h->modes.size() * slab_elem_bytes(prec);
  const size_t fit = NOALLOC_SCRATCH_BYTES / per_vec;
  if (fit == 0)
    return fail(HELIC_ERR_NOMEM, "one vector's intermediate slabs (" + std::to_string(per_vec) +
                                     " bytes) exceed the " + std::to_string(HELIC_NOALLOC_SCRATCH_MIB) +
                                     " MiB scratch array");
  const int chunk = (int)std::min<size_t>(fit, (size_t)h->dev->apply_chunk);
  LaunchSet ls = launch_set(h);
  ls.gh = ws;
  for (int v0 = 0; v0 < nvec; v0 += chunk) {
    const int nv = std::min(chunk, nvec - v0);
    const double* Xc = X + (int64_t)v0 * ldx * 2;
    double* Yc = Y + (int64_t)v0 * ldy * 2;
    const helic_status s = prec == HELIC_FP64   ? launch_stages<double>(ls, Xc, ldx, Yc, ldy, nv, st, 1, nullptr)
                           : prec == HELIC_FP32 ? launch_stages<float>(ls, Xc, ldx, Yc, ldy, nv, st, 1, nullptr)
                                                : launch_stages<bf16x2>(ls, Xc, ldx, Yc, ldy, nv, st, 1, nullptr);
    if (s != HELIC_OK) return s;
  }
  return HELIC_OK;
}

helic_status precondition_impl(helic_basis_s* h, const double* Rr, int64_t ldr, double* W, int64_t ldw,
                               int nvec, hipStream_t st) {
  DeviceState* d = h->dev;
  const int nchunk = (int)std::min<int64_t>(64, (h->L + 1023) / 1024);
  const size_t need = (size_t)nvec * nchunk * 2 * sizeof(double);
  if (need > d->part_bytes) {
    if (d->part) HIP_TRY(hipFree(d->part));
    d->part = nullptr;
    d->part_bytes = 0;
    HIP_TRY(hipMalloc((void**)&d->part, need));
    d->part_bytes = need;
  }
  hipLaunchKernelGGL(k_tpa_partial, dim3(nchunk, nvec), dim3(NT), 0, st, Rr, ldr, d->kappa, h->L, nchunk,
                     d->part);
  HIP_TRY(hipGetLastError());
  const int nb = (int)std::min<int64_t>(64, (h->L + NT - 1) / NT);
  hipLaunchKernelGGL(k_tpa_apply, dim3(nb, nvec), dim3(NT), 0, st, Rr, ldr, W, ldw, d->kappa, h->L, nchunk,
                     d->part);
  HIP_TRY(hipGetLastError());
  return HELIC_OK;
}

}  // namespace helic

using namespace helic;

extern "C" {

helic_status helic_set_potential(helic_basis h, const double* V, void* stream) {
  if (!h || !V) return fail(HELIC_ERR_INVALID, "null argument");
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  DeviceState* d = h->dev;
  const size_t n = (size_t)h->n_t1 * h->n_t2 * h->n_r;

  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int nb = (int)std::min<size_t>(4096, (n + NT - 1) / NT);
  hipLaunchKernelGGL(k_relayout_potential, dim3(nb), dim3(NT), 0, st, V, d->Vs, d->Vsf, h->n_t1, h->n_t2,
                     h->n_r, 1.0 / ((double)h->n_t1 * h->n_t2));
  HIP_TRY(hipGetLastError());
  if (d->fast_mpad) {
    const size_t nvh = (size_t)h->n_r * h->n_t2 * (2 * d->fast_mpad - 1);
    const int nbh = (int)std::min<size_t>(4096, (nvh + NT - 1) / NT);
    hipLaunchKernelGGL(k_potential_spectrum, dim3(nbh), dim3(NT), 0, st, V, d->Vh, d->Vhf, h->n_t1, h->n_t2,
                       h->n_r, d->fast_mpad);
    HIP_TRY(hipGetLastError());
  }
  // the potential's diagonal in the basis (input of the learned preconditioner)
  if (!d->vdiag) HIP_TRY(hipMalloc((void**)&d->vdiag, sizeof(double) * (h->L + h->n_r)));
  double* vbar = d->vdiag + h->L;
  hipLaunchKernelGGL(k_angular_mean, dim3(h->n_r), dim3(NT), 0, st, d->Vs, h->n_t1 * h->n_t2, vbar);
  hipLaunchKernelGGL(k_potential_diagonal, dim3((int)h->groups.size()), dim3(NT), 0, st, d->groups, d->row_ck,
                     d->tinv64, d->tfwd64, vbar, h->n_r, d->vdiag);
  HIP_TRY(hipGetLastError());
  d->have_potential = true;
  return HELIC_OK;
}

helic_status helic_apply_H(helic_basis h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                           int32_t nvec, helic_prec prec, void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!X || !Y)) || ldx < h->L || ldy < h->L)
    return fail(HELIC_ERR_INVALID, "bad block arguments");
  if (prec != HELIC_FP64 && prec != HELIC_FP32 && prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  if (nvec == 0) return HELIC_OK;
  if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "no potential set");
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  return apply_H_impl(h, X, ldx, Y, ldy, nvec, prec, reinterpret_cast<hipStream_t>(stream), APPLY_CHUNK);
}

helic_status helic_apply_H_noalloc(helic_basis h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                                   int32_t nvec, helic_prec prec, void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!X || !Y)) || ldx < h->L || ldy < h->L)
    return fail(HELIC_ERR_INVALID, "bad block arguments");
  if (prec != HELIC_FP64 && prec != HELIC_FP32 && prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  if (nvec == 0) return HELIC_OK;
  // the device state exists once a potential is set; no set-up happens here
  if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "no potential set");
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != h->dev->device) return fail(HELIC_ERR_STATE, "handle was set up on another device");
  return apply_H_noalloc_impl(h, X, ldx, Y, ldy, nvec, prec, reinterpret_cast<hipStream_t>(stream));
}

helic_status helic_profile_apply(helic_basis h, const double* X, int64_t ldx, double* Y, int64_t ldy,
                                 int32_t nvec, helic_prec prec, int32_t nrep, void* stream, double* ms_stage,
                                 double* ms_total) {
  if (!h || !ms_stage) return fail(HELIC_ERR_INVALID, "null argument");
  if (nvec <= 0 || nvec > APPLY_CHUNK || !X || !Y || ldx < h->L || ldy < h->L || nrep <= 0)
    return fail(HELIC_ERR_INVALID, "bad block arguments (1 <= nvec <= 64, nrep >= 1)");
  if (prec != HELIC_FP64 && prec != HELIC_FP32 && prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "no potential set");
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  if ((s = ensure_workspace(h, nvec, slab_elem_bytes(prec) / 2)) != HELIC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int chunk = h->dev->apply_chunk;
  const int nch = (nvec + chunk - 1) / chunk;
  // timing-only events: no system-scope fence (cache write-back and
  // invalidation) at each record, which would otherwise sit between the stages
  // start and end events of each stage kernel, carried by the kernels'
  // dispatch packets (no marker packets, no cache fences between stages)
  std::vector<hipEvent_t> ev(6 * (size_t)nrep * nch, nullptr);
  for (auto& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  for (int i = 0; i < nrep && s == HELIC_OK; ++i)
    for (int c = 0; c < nch && s == HELIC_OK; ++c) {
      const int v0 = c * chunk, nv = std::min(chunk, nvec - v0);
      hipEvent_t* e6 = &ev[6 * ((size_t)i * nch + c)];
      s = launch_apply(h, prec, X + (int64_t)v0 * ldx * 2, ldx, Y + (int64_t)v0 * ldy * 2, ldy, nv, st, 1, e6);
    }
  double acc[3] = {0, 0, 0}, tot = 0;
  if (s == HELIC_OK) {
    hipError_t e = hipStreamSynchronize(st);
    for (size_t i = 0; i < (size_t)nrep * nch && e == hipSuccess; ++i) {
      float ms;
      for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        e = hipEventElapsedTime(&ms, ev[6 * i + 2 * k], ev[6 * i + 2 * k + 1]);
        acc[k] += ms;
      }
    }
    for (int i = 0; i < nrep && e == hipSuccess; ++i) {
      float ms;
      e = hipEventElapsedTime(&ms, ev[6 * (size_t)i * nch], ev[6 * ((size_t)i * nch + nch - 1) + 5]);
      tot += ms;
    }
    if (e != hipSuccess) s = fail(HELIC_ERR_HIP, std::string("event timing: ") + hipGetErrorString(e));
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (s != HELIC_OK) return s;
  for (int k = 0; k < 3; ++k) ms_stage[k] = acc[k] / nrep;
  if (ms_total) *ms_total = tot / nrep;
  return HELIC_OK;
}

// Inverse transform of nvec columns onto nvec consecutive grids with the
// radial tables of `probs` (the basis' own, or their r-derivatives).
static helic_status inverse_transform(helic_basis_s* h, const double* X, int64_t ldx, double* g, int nvec,
                                      hipStream_t st, const DProb* probs) {
  DeviceState* d = h->dev;
  helic_status s = HELIC_OK;
  const int ng = (int)h->groups.size();
  const int64_t grid_elems = (int64_t)h->n_t1 * h->n_t2 * h->n_r;
  for (int v0 = 0; v0 < nvec; v0 += APPLY_CHUNK) {
    const int nv = std::min(APPLY_CHUNK, nvec - v0);
    if ((s = ensure_workspace(h, nv, sizeof(double))) != HELIC_OK) return s;
    double* gh = reinterpret_cast<double*>(d->gh);
    launch_radial_inverse<double>(inv_ks_for(h), 8 * ((ng * nv + 7) / 8),
                                  (size_t)h->max_kpad * lds_stride(h->max_colpad) * sizeof(double), st,
                                  X + (int64_t)v0 * ldx * 2, ldx, gh, nv, ng, h->n_r, d->groups, probs, 0);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_angular<double, 1>), dim3(8 * ((nv * h->n_r + 7) / 8)), dim3(NT),
                       angular_lds_bytes(h, sizeof(double)), st, gh, nullptr, g + v0 * grid_elems * 2, 1, nv,
                       h->n_r, probs, d->rows1, (int)h->rows1.size(), d->tw1, d->tw2, d->plan1, d->plan2, 1.0);
    HIP_TRY(hipGetLastError());
  }
  return HELIC_OK;
}

helic_status helic_transform_inverse(helic_basis h, const double* X, int64_t ldx, double* g, int32_t nvec,
                                     void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!X || !g)) || ldx < h->L) return fail(HELIC_ERR_INVALID, "bad arguments");
  if (nvec == 0) return HELIC_OK;
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  return inverse_transform(h, X, ldx, g, nvec, reinterpret_cast<hipStream_t>(stream), h->dev->probs64);
}

helic_status helic_gradient(helic_basis h, const double* X, int64_t ldx, int32_t nvec, double* grad,
                            int32_t cartesian, void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!X || !grad)) || ldx < h->L || cartesian < 0 || cartesian > 1)
    return fail(HELIC_ERR_INVALID, "bad arguments");
  if (nvec == 0) return HELIC_OK;
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  DeviceState* d = h->dev;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (!d->probs_dr) {
    // first call: d xi / dr tables, a problem entry using them, 2 pi m and
    // 2 pi n per row, the radii
    std::vector<double> fac(2 * (size_t)h->L), rg(h->n_r);
    for (int64_t i = 0; i < h->L; ++i) {
      fac[i] = 2.0 * PI_D * h->mnk[3 * i];
      fac[h->L + i] = 2.0 * PI_D * h->p.ncyc * h->mnk[3 * i + 1];   // theta2 derivative: i 2 pi N n
    }
    for (int l = 0; l < h->n_r; ++l) rg[l] = h->p.R * h->q[l];
    if (!d->tdinv64 && (s = upload(h->tab_dinv, &d->tdinv64))) return s;
    if (!d->grad_fac && (s = upload(fac, &d->grad_fac))) return s;
    if (!d->rgrid && (s = upload(rg, &d->rgrid))) return s;
    DProb p = problem_entry(h, true, 0, 0);
    p.tinv = d->tdinv64;
    std::vector<DProb> pv(1, p);
    if ((s = upload(pv, &d->probs_dr))) return s;   // set last: marks the set-up complete
  }
  const int chunk = std::min<int>(nvec, APPLY_CHUNK);
  const size_t need = (size_t)chunk * h->L * 2 * sizeof(double);
  if (need > d->grad_ws_bytes) {
    if (d->grad_ws) HIP_TRY(hipFree(d->grad_ws));
    d->grad_ws = nullptr;
    d->grad_ws_bytes = 0;
    HIP_TRY(hipMalloc((void**)&d->grad_ws, need));
    d->grad_ws_bytes = need;
  }
  const int64_t npts = (int64_t)h->n_t1 * h->n_t2 * h->n_r;
  // E_theta1, E_theta2: transforms of (i 2 pi m) x and (i 2 pi n) x
  for (int c = 0; c < 2; ++c)
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
      const int nv = std::min(chunk, nvec - v0);
      hipLaunchKernelGGL(k_scale_imag, dim3((unsigned)std::min<int64_t>(256, (h->L + NT - 1) / NT), nv), dim3(NT), 0,
                         st, X + (int64_t)v0 * ldx * 2, ldx, d->grad_ws, h->L, nv, d->grad_fac + (size_t)c * h->L);
      HIP_TRY(hipGetLastError());
      if ((s = inverse_transform(h, d->grad_ws, h->L, grad + ((int64_t)c * nvec + v0) * npts * 2, nv, st,
                                 d->probs64)))
        return s;
    }
  // E_r: the transform with d xi / dr as the radial functions
  if ((s = inverse_transform(h, X, ldx, grad + (int64_t)2 * nvec * npts * 2, nvec, st, d->probs_dr))) return s;
  if (cartesian) {
    hipLaunchKernelGGL(k_cartesian, dim3((unsigned)std::min<int64_t>(1024, (npts + NT - 1) / NT), nvec), dim3(NT), 0,
                       st, grad, nvec, h->n_t1, h->n_t2, h->n_r, d->rgrid, h->p.alpha, h->p.tau, h->p.ncyc);
    HIP_TRY(hipGetLastError());
  }
  return HELIC_OK;
}

helic_status helic_transform_forward(helic_basis h, const double* g, double* X, int64_t ldx, int32_t nvec,
                                     void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!X || !g)) || ldx < h->L) return fail(HELIC_ERR_INVALID, "bad arguments");
  if (nvec == 0) return HELIC_OK;
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  DeviceState* d = h->dev;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int ng = (int)h->groups.size();
  const int64_t grid_elems = (int64_t)h->n_t1 * h->n_t2 * h->n_r;
  for (int v0 = 0; v0 < nvec; v0 += APPLY_CHUNK) {
    const int nv = std::min(APPLY_CHUNK, nvec - v0);
    if ((s = ensure_workspace(h, nv, sizeof(double))) != HELIC_OK) return s;
    double* gh = reinterpret_cast<double*>(d->gh);
    hipLaunchKernelGGL((k_angular<double, 2>), dim3(8 * ((nv * h->n_r + 7) / 8)), dim3(NT),
                       angular_lds_bytes(h, sizeof(double)), st, gh, g + v0 * grid_elems * 2, nullptr, 1, nv,
                       h->n_r, d->probs64, d->rows1, (int)h->rows1.size(), d->tw1, d->tw2, d->plan1, d->plan2,
                       1.0 / ((double)h->n_t1 * h->n_t2));
    HIP_TRY(hipGetLastError());
    launch_radial_forward<double>(4, 8 * ((ng * nv + 7) / 8),
                                  fwd_lds_bytes(h, sizeof(double)), st, gh, (const double*)nullptr, ldx,
                                  X + (int64_t)v0 * ldx * 2, ldx, nv, ng, h->n_r, d->groups, d->probs64, 0, 0);
    HIP_TRY(hipGetLastError());
  }
  return HELIC_OK;
}

helic_status helic_density(helic_basis h, const double* X, int64_t ldx, int32_t nvec, const double* occ,
                           double* rho, int32_t accumulate, void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!X || !occ)) || !rho || ldx < h->L) return fail(HELIC_ERR_INVALID, "bad arguments");
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  DeviceState* d = h->dev;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t npts = (int64_t)h->n_t1 * h->n_t2 * h->n_r;
  const unsigned nb = (unsigned)std::min<int64_t>(4096, (npts + NT - 1) / NT);
  if (nvec == 0) {
    if (!accumulate) {
      hipLaunchKernelGGL(k_density_accum, dim3(nb), dim3(NT), 0, st, (const double*)nullptr, 0, npts,
                         (const double*)nullptr, rho, 0);
      HIP_TRY(hipGetLastError());
    }
    return HELIC_OK;
  }
  const int chunk = std::min(nvec, DENSITY_CHUNK);
  const size_t need = (size_t)chunk * npts * 2 * sizeof(double);
  if (need > d->dens_ws_bytes) {
    if (d->dens_ws) HIP_TRY(hipFree(d->dens_ws));
    d->dens_ws = nullptr;
    d->dens_ws_bytes = 0;
    HIP_TRY(hipMalloc((void**)&d->dens_ws, need));
    d->dens_ws_bytes = need;
  }
  if ((size_t)nvec > d->dens_occ_n) {
    if (d->dens_occ) HIP_TRY(hipFree(d->dens_occ));
    d->dens_occ = nullptr;
    d->dens_occ_n = 0;
    HIP_TRY(hipMalloc((void**)&d->dens_occ, sizeof(double) * nvec));
    d->dens_occ_n = nvec;
  }
  HIP_TRY(hipMemcpyAsync(d->dens_occ, occ, sizeof(double) * nvec, hipMemcpyHostToDevice, st));
  for (int v0 = 0; v0 < nvec; v0 += chunk) {
    const int nv = std::min(chunk, nvec - v0);
    if ((s = helic_transform_inverse(h, X + (int64_t)v0 * ldx * 2, ldx, d->dens_ws, nv, stream)) != HELIC_OK)
      return s;
    hipLaunchKernelGGL(k_density_accum, dim3(nb), dim3(NT), 0, st, d->dens_ws, nv, npts, d->dens_occ + v0, rho,
                       (v0 > 0 || accumulate) ? 1 : 0);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  return HELIC_OK;
}

helic_status helic_precondition(helic_basis h, const double* Rres, int64_t ldr, double* W, int64_t ldw,
                                int32_t nvec, void* stream) {
  if (!h) return fail(HELIC_ERR_INVALID, "null handle");
  if (nvec < 0 || (nvec > 0 && (!Rres || !W)) || ldr < h->L || ldw < h->L)
    return fail(HELIC_ERR_INVALID, "bad block arguments");
  if (nvec == 0) return HELIC_OK;
  if (W != Rres) {
    // W may equal R (in place) but must not partially overlap it
    const char* a = reinterpret_cast<const char*>(Rres);
    const char* b = reinterpret_cast<const char*>(W);
    const size_t na = (size_t)ldr * nvec * 16, nb = (size_t)ldw * nvec * 16;
    if (a < b + nb && b < a + na) return fail(HELIC_ERR_INVALID, "R and W overlap");
  } else if (ldr != ldw) {
    return fail(HELIC_ERR_INVALID, "in-place preconditioning needs ldr == ldw");
  }
  helic_status s = ensure_device(h);
  if (s != HELIC_OK) return s;
  return precondition_impl(h, Rres, ldr, W, ldw, nvec, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
