// Radial stages of H*X in the BF16 mode: the contractions of Alg. 1 and Alg. 3
// (radial parts) on 16x16x16 BF16 MFMA with FP32 accumulation, reading and
// writing the intermediate slabs as bfloat16 pairs (bf16x2).  Same work split
// as the FP64/FP32 kernels (one |n| group x one vector per workgroup, vector-
// major XCD mapping); the tables are the basis' BF16 copies, whose fragments
// hold 16 rows x 16 contraction indices (lane l: row l % 16, contraction
// indices 4 (l / 16) + 0..3).  Included by device.hip after the helpers it
// shares with the other radial kernels (tile_kmax, swap_lane_pairs).
#pragma once
#include "kernels.hpp"

namespace helic {

// LDS stride (bfloat16 elements) of one staged column: 8 beyond a multiple of
// 16, so the 16 columns an MFMA operand reads (8 bytes per lane) start on
// distinct LDS banks.
__host__ __device__ constexpr int bf16_col_stride(int len16) { return len16 + 8; }
constexpr int FWD16_RC = 16;   // radii staged per chunk of the forward kernel
constexpr int FWD16_COLS = 256; // widest staged group (real columns) the forward kernel takes

// G_{mn}(r_l) = sum_k xi_{|n|,k}(r_l) x_{mnk}: the group's coefficients are
// staged in LDS as bfloat16 columns [2 modes][k] (re and im as separate real
// columns, k contiguous, zero beyond each mode's K); each wave takes 16-radius
// tiles; KT16 bounds the k steps (of 16) of the widest group.
template <int KT16>
__global__ void __launch_bounds__(NT)
k_radial_inverse_bf16(const double* __restrict__ X, int64_t ldx, bf16x2* __restrict__ GH, int nvec, int ngroups,
                      int n_r, const DGroup* __restrict__ groups, const DProb* __restrict__ probs, int order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t* Bs = reinterpret_cast<uint16_t*>(smem_raw);
  int v, gi;
  if (!radial_item(order, ngroups, nvec, v, gi)) return;
  const DGroup gr = groups[gi];
  const DProb& pb = probs[gr.prob];
  const int nk16 = (gr.Kmax + 15) / 16;
  const int kst = bf16_col_stride(16 * nk16);
  const int ncol = 2 * gr.nmodes;
  const int nct = (ncol + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nrt = (n_r + 15) / 16;
  uint32_t* Bw = reinterpret_cast<uint32_t*>(Bs);
  for (int i = threadIdx.x; i < 16 * nct * kst / 2; i += NT) Bw[i] = 0u;
  __syncthreads();
  const double2* xv = reinterpret_cast<const double2*>(X + col_off(pb, ldx, nvec, v) * 2) + gr.row0;
  for (int i = threadIdx.x; i < (int)gr.nrows; i += NT) {
    const int ck = pb.row_ck[gr.row0 + i];
    const int c = ck >> 16, k = ck & 0xffff;
    const double2 x = xv[i];
    Bs[(2 * c) * kst + k] = (uint16_t)bf16_bits((float)x.x);
    Bs[(2 * c + 1) * kst + k] = (uint16_t)bf16_bits((float)x.y);
  }
  __syncthreads();
  const uint64_t* tg = reinterpret_cast<const uint64_t*>(pb.tinv) + gr.tinv16_off;
  bf16x2* gv = GH + slab_off(pb, nvec, n_r, v, 0) + gr.mode0;
  // k steps of column tile c: lane c holds the largest K of the tile's modes
  const int ktile = tile_kmax(pb.modes + gr.mode0, gr.nmodes, lane);
  const int bpos = (lane & 15) * kst + 4 * (lane >> 4);
  for (int rt = wave; rt < nrt; rt += NT / 64) {
    uint64_t a[KT16];
#pragma unroll
    for (int s = 0; s < KT16; ++s) a[s] = s < nk16 ? tg[((int64_t)rt * nk16 + s) * 64 + lane] : 0ull;
    for (int ct = 0; ct < nct; ++ct) {
      const int ks = nct <= 64 ? (__builtin_amdgcn_readlane(ktile, ct) + 15) / 16 : nk16;
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
      const uint16_t* bt = Bs + 16 * ct * kst + bpos;
#pragma unroll
      for (int s = 0; s < KT16; ++s)
        if (s < ks) acc = mfma_bf16(a[s], *reinterpret_cast<const uint64_t*>(bt + 16 * s), acc);
      // lanes 2j and 2j + 1 hold re and im of one mode for the same radii;
      // after a swap across the pair each lane stores two complex values
      float sw[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) sw[i] = swap_lane_pairs(acc[i]);
      const int col = 16 * ct + (lane & 15);
      if (col < ncol) {
        const bool odd = lane & 1;
        bf16x2* dst = gv + (col >> 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = odd ? 2 * h + 1 : 2 * h;
          const int r = 16 * rt + 4 * (lane >> 4) + i;
          const float re = odd ? sw[i] : acc[i];
          const float im = odd ? acc[i] : sw[i];
          if (r < n_r) estore<float>(dst + (int64_t)r * pb.n_modes, cplx<float>{re, im});
        }
      }
    }
  }
}

// y_{mnk} = kappa x_{mnk} + sum_l (2 pi tau omega_l xi_{|n|,k}(r_l)) H_{mn}(r_l):
// chunks of FWD16_RC radii of the group's slab rows are staged in LDS as
// bfloat16 columns [2 modes][r] (r contiguous, one 8-byte word per four radii
// of a real column), together with the chunk's table fragments of every k
// tile; the next chunk is fetched into registers while the MFMAs of the
// current one run.  Each wave accumulates up to TM output tiles over all
// chunks, then adds kappa x in FP64 and writes rows k <= K of each mode.
// LDS: colpad x FWD16_RC bfloat16 (+ padding) and 6 x 2 fragments of 512 B.
constexpr int FWD16_KT = 6;                                   // k tiles (of 16) per group it supports
constexpr int FWD16_CST = FWD16_RC / 4 + 2;                   // column stride in 8-byte words
constexpr int FWD16_QMAX = 2;                                 // staged (mode, radius quad) items per thread
__host__ __device__ constexpr size_t fwd16_table_off(int colpad) {
  return ((size_t)colpad * FWD16_CST * 8 + 15) & ~(size_t)15;
}

template <int TM>
__global__ void __launch_bounds__(NT)
k_radial_forward_bf16(const bf16x2* __restrict__ GH, const double* __restrict__ X, int64_t ldx,
                      double* __restrict__ Y, int64_t ldy, int nvec, int ngroups, int n_r,
                      const DGroup* __restrict__ groups, const DProb* __restrict__ probs, int add_kinetic,
                      int order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int RQ = FWD16_RC / 4;             // radius quads per chunk
  constexpr int RS = FWD16_RC / 16;            // MFMA k steps per chunk
  uint64_t* Hs = reinterpret_cast<uint64_t*>(smem_raw);
  int v, gi;
  if (!radial_item(order, ngroups, nvec, v, gi)) return;
  const DGroup gr = groups[gi];
  const DProb& pb = probs[gr.prob];
  const int nmodes = gr.nmodes;
  const int ncol = 2 * nmodes;
  const int nct = (ncol + 15) / 16;
  const int half = 8 * nct;   // staged (re, im) column pairs, padded to whole tiles
  const int nkt = (gr.Kmax + 15) / 16;
  const int ntiles = nkt * nct;
  const int nr16 = (n_r + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t* As = reinterpret_cast<uint64_t*>(smem_raw + fwd16_table_off(16 * nct));   // [kt][s][64]
  const uint64_t* tg = reinterpret_cast<const uint64_t*>(pb.tfwd) + gr.tfwd16_off;
  const bf16x2* hv = GH + slab_off(pb, nvec, n_r, v, 0) + gr.mode0;
  const DMode* modes = pb.modes;
  const double* kappa = pb.kappa;
  const double* xv = add_kinetic ? X + col_off(pb, ldx, nvec, v) * 2 : nullptr;
  double* yv = Y + col_off(pb, ldy, nvec, v) * 2;
  const int ktile = tile_kmax(modes + gr.mode0, nmodes, lane);
  const int nitems = half * RQ;                // (mode, radius quad) pairs of a chunk
  const int nfrag = nkt * RS * 64;             // table fragment words of a chunk
  uint64_t re4[FWD16_QMAX], im4[FWD16_QMAX], ta[(FWD16_KT * RS * 64 + NT - 1) / NT];
  // item i = (quad q, mode c), modes fastest: coalesced 4-byte reads
  auto fetch = [&](int r0) {
#pragma unroll
    for (int a = 0; a < FWD16_QMAX; ++a) {
      const int i = threadIdx.x + NT * a;
      uint32_t u[4] = {0u, 0u, 0u, 0u};
      if (i < nitems) {
        const int q = i / half, c = i - q * half;
        if (c < nmodes) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * q + j;
            if (r < n_r) u[j] = hv[(int64_t)r * pb.n_modes + c].u;
          }
        }
      }
      re4[a] = (uint64_t)(u[0] & 0xffffu) | ((uint64_t)(u[1] & 0xffffu) << 16) |
               ((uint64_t)(u[2] & 0xffffu) << 32) | ((uint64_t)(u[3] & 0xffffu) << 48);
      im4[a] = (uint64_t)(u[0] >> 16) | ((uint64_t)(u[1] >> 16) << 16) | ((uint64_t)(u[2] >> 16) << 32) |
               ((uint64_t)(u[3] >> 16) << 48);
    }
    const int rs0 = r0 / 16;
#pragma unroll
    for (int a = 0; a < (FWD16_KT * RS * 64 + NT - 1) / NT; ++a) {
      const int i = threadIdx.x + NT * a;
      uint64_t w = 0ull;
      if (i < nfrag) {
        const int ln = i & 63, ks = i >> 6;
        const int kt = ks / RS, s = ks - kt * RS;
        if (rs0 + s < nr16) w = tg[((int64_t)kt * nr16 + rs0 + s) * 64 + ln];
      }
      ta[a] = w;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int a = 0; a < FWD16_QMAX; ++a) {
      const int i = threadIdx.x + NT * a;
      if (i < nitems) {
        const int q = i / half, c = i - q * half;
        Hs[(2 * c) * FWD16_CST + q] = re4[a];
        Hs[(2 * c + 1) * FWD16_CST + q] = im4[a];
      }
    }
#pragma unroll
    for (int a = 0; a < (FWD16_KT * RS * 64 + NT - 1) / NT; ++a) {
      const int i = threadIdx.x + NT * a;
      if (i < nfrag) As[i] = ta[a];
    }
  };
  const int nchunk = (n_r + FWD16_RC - 1) / FWD16_RC;
  for (int tbase = 0; tbase < ntiles; tbase += (NT / 64) * TM) {
    f32x4_t acc[TM];
    int tk[TM], tc[TM];
    bool live[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      acc[i] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      const int t = tbase + wave + (NT / 64) * i;
      tk[i] = t / nct;
      tc[i] = t - tk[i] * nct;
      live[i] = t < ntiles && (nct > 64 || 16 * tk[i] < __builtin_amdgcn_readlane(ktile, tc[i]));
    }
    fetch(0);
    for (int ch = 0; ch < nchunk; ++ch) {
      __syncthreads();
      store();
      __syncthreads();
      if (ch + 1 < nchunk) fetch((ch + 1) * FWD16_RC);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        if (!live[i]) continue;
        const uint64_t* bt = Hs + (16 * tc[i] + (lane & 15)) * FWD16_CST + (lane >> 4);
#pragma unroll
        for (int s = 0; s < RS; ++s)
          acc[i] = mfma_bf16(As[(tk[i] * RS + s) * 64 + lane], bt[4 * s], acc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      if (!live[i]) continue;
      const int col = 16 * tc[i] + (lane & 15);
      const int c = col >> 1, ri = col & 1;
      if (c >= nmodes) continue;
      const DMode md = modes[gr.mode0 + c];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * tk[i] + 4 * (lane >> 4) + j;
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

}  // namespace helic
