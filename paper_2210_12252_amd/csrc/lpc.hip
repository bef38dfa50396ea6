// Learned diagonal preconditioner: per-coefficient MLP scale s_ij applied to
// the LOBPCG residuals, its training kernels (forward, direction loss,
// backward with per-workgroup partial gradients reduced in a fixed order,
// Adam) and the C-ABI around them.  The paper has no learned component; the
// network refines the Teter-Payne-Allan factor of Sec. 3.5, which it equals
// when its last layer is zero.
//
// Work layout: one thread per coefficient (row i of column j).  Features and
// column statistics are FP64, the network runs in FP32 with its parameters
// staged in LDS (broadcast reads), the correction is written in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "device_state.hpp"
#include "helic_internal.h"

struct helic_lpc_s {
  int device = 0;
  float* theta = nullptr;   // parameters (NPAD floats, tail zero)
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  double* grad = nullptr;   // last gradient (NPARAM)
  float* gpart = nullptr;   // per-workgroup partial gradients
  size_t gpart_bytes = 0;
  int32_t* tidx = nullptr;  // training: column indices of the current batch
  int tidx_n = 0;
  int step = 0;
};

namespace helic {

helic_status precondition_impl(helic_basis_s* h, const double* Rr, int64_t ldr, double* W, int64_t ldw,
                               int nvec, hipStream_t st);

namespace {

constexpr int NIN = 8, HID = 64;
constexpr int P_W1 = 0, P_B1 = P_W1 + HID * NIN, P_W2 = P_B1 + HID, P_B2 = P_W2 + HID * HID, P_W3 = P_B2 + HID,
              P_B3 = P_W3 + HID, NPARAM = P_B3 + 1;
static_assert(NPARAM == HELIC_LPC_NPARAM, "parameter layout");
constexpr int NPAD = (NPARAM + 3) / 4 * 4;
constexpr int LT = 256;            // threads per workgroup = coefficients per tile
constexpr int NREM = 2 * HID + HID + 1;   // b1, b2, w3, b3: 193 entries owned one per thread
constexpr float INV_LOG2 = 1.4426950408889634f;

#define HIP_TRY_L(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(HELIC_ERR_HIP, std::string(#call) + " (lpc line " + std::to_string(__LINE__) + "): " + \
                                     hipGetErrorString(e_));                         \
  } while (0)

// Per-column record: TPA energy T, residual norm, Ritz value, and for
// training <s r, t>, ||s r||^2, ||t||^2 and the column's loss.
struct ColRec {
  double T, rn, lam, are, aim, B, C, loss;
};

__device__ inline float silu(float x) { return x / (1.0f + __expf(-x)); }
__device__ inline float dsilu(float x) {
  const float sg = 1.0f / (1.0f + __expf(-x));
  return sg * (1.0f + x * (1.0f - sg));
}
__device__ inline float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(__expf(-fabsf(x))); }

__device__ inline void stage_params(const float* __restrict__ theta, float* sw) {
  for (int i = threadIdx.x; i < NPAD; i += blockDim.x) sw[i] = theta[i];
}

// Features of one coefficient and its TPA factor.
__device__ inline void features(double kap, double vd, double re, double im, const ColRec& c, double sqrtL,
                                float* f, float* K) {
  const double g = kap / c.T;
  const double num = 27.0 + g * (18.0 + g * (12.0 + 8.0 * g));
  const double k = num / (num + 16.0 * g * g * g * g);
  *K = (float)k;
  f[0] = (float)k;
  f[1] = (float)log(g);
  f[2] = (float)log(kap);
  f[3] = (float)((vd - c.lam) / c.T);
  f[4] = (float)(c.lam / c.T);
  f[5] = (float)log(sqrt(re * re + im * im) * sqrtL / c.rn + 1e-30);
  f[6] = 0.0f;
  f[7] = 0.0f;
}

// First layer: h1 = silu(W1 f + b1).
__device__ inline void layer1(const float* sw, const float* f, float* h1) {
#pragma unroll
  for (int k = 0; k < HID; ++k) {
    float a = sw[P_B1 + k];
#pragma unroll
    for (int q = 0; q < NIN; ++q) a = fmaf(sw[P_W1 + k * NIN + q], f[q], a);
    h1[k] = silu(a);
  }
}

// Scale of one coefficient (inference: layer 2 outputs are not kept).
__device__ inline float mlp_scale(const float* sw, const float* f, float K) {
  float h1[HID];
  layer1(sw, f, h1);
  float z = sw[P_B3];
  for (int o = 0; o < HID; ++o) {
    const float* w2 = sw + P_W2 + o * HID;
    float a = sw[P_B2 + o];
#pragma unroll
    for (int k = 0; k < HID; ++k) a = fmaf(w2[k], h1[k], a);
    z = fmaf(sw[P_W3 + o], silu(a), z);
  }
  return K * softplus(z) * INV_LOG2;
}

__device__ inline int col_of(const int32_t* cidx, int j) { return cidx ? cidx[j] : j; }

// Column partial sums over row blocks: |r|^2, kappa |r|^2, |t|^2.
__global__ void __launch_bounds__(LT)
k_col_partial(const double* __restrict__ R, int64_t ldr, const double* __restrict__ Tt, int64_t ldt,
              const int32_t* __restrict__ cidx, const double* __restrict__ kappa, int64_t L,
              double* __restrict__ part) {
  __shared__ double red[3][LT];
  const int j = blockIdx.y, nb = gridDim.x;
  const int jc = col_of(cidx, j);
  const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  if (i < L) {
    const double* r = R + ((int64_t)jc * ldr + i) * 2;
    const double m2 = r[0] * r[0] + r[1] * r[1];
    a = m2;
    b = kappa[i] * m2;
    if (Tt) {
      const double* t = Tt + ((int64_t)jc * ldt + i) * 2;
      c = t[0] * t[0] + t[1] * t[1];
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int w = LT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[((int64_t)j * nb + blockIdx.x) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Column records from the partial sums (fixed order: deterministic).  A zero
// column gets T = 1, rn = 1 (its correction is zero whatever s is).
__global__ void k_col_finish(const double* __restrict__ part, int nb, int ncol, const double* __restrict__ lam,
                             const int32_t* __restrict__ cidx, ColRec* __restrict__ cols) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int q = 0; q < nb; ++q) {
    a += part[((int64_t)j * nb + q) * 3];
    b += part[((int64_t)j * nb + q) * 3 + 1];
    c += part[((int64_t)j * nb + q) * 3 + 2];
  }
  ColRec r{};
  const bool zero = !(a > 0.0);
  r.T = zero ? 1.0 : b / a;
  r.rn = zero ? 1.0 : sqrt(a);
  r.lam = lam[col_of(cidx, j)];
  r.C = c;
  cols[j] = r;
}

// Inference: W = s R.
__global__ void __launch_bounds__(LT)
k_lpc_apply(const double* __restrict__ R, int64_t ldr, double* __restrict__ W, int64_t ldw,
            const double* __restrict__ kappa, const double* __restrict__ vdiag, int64_t L, double sqrtL,
            const ColRec* __restrict__ cols, const float* __restrict__ theta) {
  __shared__ float sw[NPAD];
  stage_params(theta, sw);
  __syncthreads();
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (i >= L) return;
  const ColRec c = cols[j];
  const double* r = R + ((int64_t)j * ldr + i) * 2;
  const double re = r[0], im = r[1];
  float f[NIN], K;
  features(kappa[i], vdiag[i], re, im, c, sqrtL, f, &K);
  const double s = (double)mlp_scale(sw, f, K);
  double* w = W + ((int64_t)j * ldw + i) * 2;
  w[0] = s * re;
  w[1] = s * im;
}

// Training forward: partial sums of <s r, t> and ||s r||^2 per row block.
__global__ void __launch_bounds__(LT)
k_lpc_fwd_partial(const double* __restrict__ R, int64_t ldr, const double* __restrict__ Tt, int64_t ldt,
                  const int32_t* __restrict__ cidx, const double* __restrict__ kappa,
                  const double* __restrict__ vdiag, int64_t L, double sqrtL, const ColRec* __restrict__ cols,
                  const float* __restrict__ theta, double* __restrict__ part) {
  __shared__ float sw[NPAD];
  __shared__ double red[3][LT];
  stage_params(theta, sw);
  __syncthreads();
  const int j = blockIdx.y, nb = gridDim.x;
  const int jc = col_of(cidx, j);
  const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
  double are = 0.0, aim = 0.0, b = 0.0;
  if (i < L) {
    const ColRec c = cols[j];
    const double* r = R + ((int64_t)jc * ldr + i) * 2;
    const double* t = Tt + ((int64_t)jc * ldt + i) * 2;
    float f[NIN], K;
    features(kappa[i], vdiag[i], r[0], r[1], c, sqrtL, f, &K);
    const double s = (double)mlp_scale(sw, f, K);
    // s conj(r) t
    are = s * (r[0] * t[0] + r[1] * t[1]);
    aim = s * (r[0] * t[1] - r[1] * t[0]);
    b = s * s * (r[0] * r[0] + r[1] * r[1]);
  }
  red[0][threadIdx.x] = are;
  red[1][threadIdx.x] = aim;
  red[2][threadIdx.x] = b;
  __syncthreads();
  for (int w = LT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[((int64_t)j * nb + blockIdx.x) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Column loss 1 - |A|^2 / (B C); columns with B or C zero contribute zero.
__global__ void k_loss_finish(const double* __restrict__ part, int nb, int ncol, ColRec* __restrict__ cols) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  double are = 0.0, aim = 0.0, b = 0.0;
  for (int q = 0; q < nb; ++q) {
    are += part[((int64_t)j * nb + q) * 3];
    aim += part[((int64_t)j * nb + q) * 3 + 1];
    b += part[((int64_t)j * nb + q) * 3 + 2];
  }
  ColRec& c = cols[j];
  c.are = are;
  c.aim = aim;
  c.B = b;
  c.loss = (b > 0.0 && c.C > 0.0) ? 1.0 - (are * are + aim * aim) / (b * c.C) : 0.0;
}

// Position of entry k of staged row e: rows of 64 floats, 4-float chunks
// rotated by the row index so that a wave writing its rows (one per lane)
// and a wave reading one row both stay free of bank conflicts.
__device__ inline int swz(int e, int k) { return e * HID + ((((k >> 2) ^ (e & 15)) << 2) | (k & 3)); }

// Training backward.  Each workgroup walks tiles of LT coefficients (column-
// major over the nvec columns), recomputes the forward pass, forms dloss/dz
// per coefficient and accumulates the parameter gradient: the W2 block
// (outer products of dloss/da2 and h1 over the tile) in registers, 4 x 4
// entries per thread; W1 two entries and one of b1/b2/w3/b3 per thread.
// Each thread keeps its coefficient's layer-2 values in its own LDS row, so
// only one 64-vector (h1, then dloss/dh1) lives in registers.  Each
// workgroup writes its partial gradient.
__global__ void __launch_bounds__(LT)
k_lpc_backward(const double* __restrict__ R, int64_t ldr, const double* __restrict__ Tt, int64_t ldt,
               const int32_t* __restrict__ cidx, const double* __restrict__ kappa,
               const double* __restrict__ vdiag, int64_t L, int ncol, double sqrtL,
               const ColRec* __restrict__ cols, const float* __restrict__ theta, float* __restrict__ gpart,
               int64_t ntiles) {
  extern __shared__ float lds[];
  float* sw = lds;                  // parameters
  float* Ah = sw + NPAD;            // [LT][HID]: h1, later dloss/da1
  float* Ab = Ah + LT * HID;        // [LT][HID]: a2, later dloss/da2
  float* AF = Ab + LT * HID;        // [LT][NIN]: features
  float* Adz = AF + LT * NIN;       // [LT]: dloss/dz
  stage_params(theta, sw);
  __syncthreads();
  const int t = threadIdx.x;
  const int o0 = 4 * (t >> 4), k0 = 4 * (t & 15);
  float g2[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) g2[q] = 0.0f;
  float gw1a = 0.0f, gw1b = 0.0f, grem = 0.0f;
  const int64_t total = L * (int64_t)ncol;
  const float inv_ncol = 1.0f / (float)ncol;

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e = tile * LT + t;
    float f[NIN], h[HID];
    float dz = 0.0f;
#pragma unroll
    for (int q = 0; q < NIN; ++q) f[q] = 0.0f;
#pragma unroll
    for (int k = 0; k < HID; ++k) h[k] = 0.0f;
    if (e < total) {
      const int j = (int)(e / L);
      const int64_t i = e - (int64_t)j * L;
      const int jc = col_of(cidx, j);
      const ColRec c = cols[j];
      const double* r = R + ((int64_t)jc * ldr + i) * 2;
      const double* tt = Tt + ((int64_t)jc * ldt + i) * 2;
      float K;
      features(kappa[i], vdiag[i], r[0], r[1], c, sqrtL, f, &K);
      layer1(sw, f, h);
      float z = sw[P_B3];
      for (int o = 0; o < HID; ++o) {
        const float* w2 = sw + P_W2 + o * HID;
        float a = sw[P_B2 + o];
#pragma unroll
        for (int k = 0; k < HID; ++k) a = fmaf(w2[k], h[k], a);
        Ab[swz(t, o)] = a;
        z = fmaf(sw[P_W3 + o], silu(a), z);
      }
      if (c.B > 0.0 && c.C > 0.0) {
        const double s = (double)(K * softplus(z) * INV_LOG2);
        const double m2 = r[0] * r[0] + r[1] * r[1];
        // d|A|^2/ds = 2 Re(conj(A) conj(r) t); dB/ds = 2 s |r|^2
        const double crt_re = r[0] * tt[0] + r[1] * tt[1], crt_im = r[0] * tt[1] - r[1] * tt[0];
        const double dA = 2.0 * (c.are * crt_re + c.aim * crt_im);
        const double A2 = c.are * c.are + c.aim * c.aim;
        const double ds = -(dA * c.B - A2 * 2.0 * s * m2) / (c.B * c.B * c.C);
        const float sg = 1.0f / (1.0f + __expf(-z));
        dz = (float)ds * inv_ncol * K * INV_LOG2 * sg;
      }
    } else {
      for (int o = 0; o < HID; ++o) Ab[swz(t, o)] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < HID; k += 4)
      *reinterpret_cast<float4*>(Ah + swz(t, k)) = make_float4(h[k], h[k + 1], h[k + 2], h[k + 3]);
#pragma unroll
    for (int q = 0; q < NIN; ++q) AF[t * NIN + q] = f[q];
    Adz[t] = dz;
    __syncthreads();
    if (t >= 2 * HID && t < 3 * HID) {          // w3: sum of dz * h2
      const int o = t - 2 * HID;
      float acc = 0.0f;
      for (int ee = 0; ee < LT; ++ee) acc = fmaf(Adz[ee], silu(Ab[swz(ee, o)]), acc);
      grem += acc;
    } else if (t == 3 * HID) {                  // b3
      float acc = 0.0f;
      for (int ee = 0; ee < LT; ++ee) acc += Adz[ee];
      grem += acc;
    }
    __syncthreads();
    for (int o = 0; o < HID; ++o) {             // own row: a2 -> dloss/da2
      const int q = swz(t, o);
      Ab[q] = dz * sw[P_W3 + o] * dsilu(Ab[q]);
    }
    __syncthreads();
    if (t >= HID && t < 2 * HID) {              // b2
      const int o = t - HID;
      float acc = 0.0f;
      for (int ee = 0; ee < LT; ++ee) acc += Ab[swz(ee, o)];
      grem += acc;
    }
    for (int ee = 0; ee < LT; ++ee) {           // W2 block
      const float4 da = *reinterpret_cast<const float4*>(Ab + swz(ee, o0));
      const float4 hh = *reinterpret_cast<const float4*>(Ah + swz(ee, k0));
      const float dv[4] = {da.x, da.y, da.z, da.w}, hv[4] = {hh.x, hh.y, hh.z, hh.w};
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) g2[p * 4 + q] = fmaf(dv[p], hv[q], g2[p * 4 + q]);
    }
    // dloss/da1 = (W2^T dloss/da2) * silu'(a1), into h
#pragma unroll
    for (int k = 0; k < HID; ++k) h[k] = 0.0f;
    for (int o = 0; o < HID; ++o) {
      const float d2 = Ab[swz(t, o)];
      const float* w2 = sw + P_W2 + o * HID;
#pragma unroll
      for (int k = 0; k < HID; ++k) h[k] = fmaf(d2, w2[k], h[k]);
    }
#pragma unroll
    for (int k = 0; k < HID; ++k) {
      float a = sw[P_B1 + k];
#pragma unroll
      for (int q = 0; q < NIN; ++q) a = fmaf(sw[P_W1 + k * NIN + q], f[q], a);
      h[k] *= dsilu(a);
    }
    __syncthreads();                            // reads of h1 and dloss/da2 done
#pragma unroll
    for (int k = 0; k < HID; k += 4)
      *reinterpret_cast<float4*>(Ah + swz(t, k)) = make_float4(h[k], h[k + 1], h[k + 2], h[k + 3]);
    __syncthreads();
    {                                           // W1 (entries t and t + LT)
      const int ka = t >> 3, kb = (t + LT) >> 3, q = t & 7;
      float acc_a = 0.0f, acc_b = 0.0f;
      for (int ee = 0; ee < LT; ++ee) {
        const float x = AF[ee * NIN + q];
        acc_a = fmaf(Ah[swz(ee, ka)], x, acc_a);
        acc_b = fmaf(Ah[swz(ee, kb)], x, acc_b);
      }
      gw1a += acc_a;
      gw1b += acc_b;
    }
    if (t < HID) {                              // b1
      float acc = 0.0f;
      for (int ee = 0; ee < LT; ++ee) acc += Ah[swz(ee, t)];
      grem += acc;
    }
    __syncthreads();
  }
  float* gp = gpart + (int64_t)blockIdx.x * NPAD;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) gp[P_W2 + (o0 + p) * HID + k0 + q] = g2[p * 4 + q];
  gp[P_W1 + t] = gw1a;
  gp[P_W1 + t + LT] = gw1b;
  if (t < HID) gp[P_B1 + t] = grem;
  else if (t < 2 * HID) gp[P_B2 + t - HID] = grem;
  else if (t < 3 * HID) gp[P_W3 + t - 2 * HID] = grem;
  else if (t == 3 * HID) gp[P_B3] = grem;
}
static_assert(2 * LT == HID * NIN, "W1 ownership: two entries per thread");
static_assert(NREM <= LT, "one remaining entry per thread");

__global__ void k_grad_reduce(const float* __restrict__ gpart, int nwg, double* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  double acc = 0.0;
  for (int w = 0; w < nwg; ++w) acc += (double)gpart[(int64_t)w * NPAD + p];
  grad[p] = acc;
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const double* __restrict__ grad, float lr, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = (float)grad[p];
  const float mm = 0.9f * m[p] + 0.1f * g;
  const float vv = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

constexpr size_t BWD_LDS = (size_t)(NPAD + 2 * LT * HID + LT * NIN + LT) * sizeof(float);

// ---- host side ----------------------------------------------------------

helic_status check_net(const helic_lpc_s* net) {
  int dev = 0;
  HIP_TRY_L(hipGetDevice(&dev));
  if (dev != net->device) return fail(HELIC_ERR_INVALID, "network lives on another device");
  return HELIC_OK;
}

// Per-call column workspace of a basis: partial sums and records.
helic_status column_ws(helic_basis_s* h, int ncol, int nb, double** part, ColRec** cols) {
  DeviceState* d = h->dev;
  const size_t np = (size_t)ncol * nb * 3;
  const size_t need = np * sizeof(double) + (size_t)ncol * sizeof(ColRec);
  if (need > d->lpc_ws_bytes) {
    if (d->lpc_ws) HIP_TRY_L(hipFree(d->lpc_ws));
    d->lpc_ws = nullptr;
    d->lpc_ws_bytes = 0;
    HIP_TRY_L(hipMalloc((void**)&d->lpc_ws, need));
    d->lpc_ws_bytes = need;
  }
  *part = d->lpc_ws;
  *cols = reinterpret_cast<ColRec*>(d->lpc_ws + np);
  return HELIC_OK;
}

helic_status ready(helic_basis_s* h) {
  if (!h->dev || !h->dev->have_potential || !h->dev->vdiag) return fail(HELIC_ERR_STATE, "no potential set");
  return HELIC_OK;
}

helic_status column_records(helic_basis_s* h, const double* R, int64_t ldr, const double* T, int64_t ldt,
                            const int32_t* cidx, const double* lam, int ncol, hipStream_t st, double** part,
                            ColRec** cols, int* nb_out) {
  const int nb = (int)((h->L + LT - 1) / LT);
  helic_status s = column_ws(h, ncol, nb, part, cols);
  if (s) return s;
  hipLaunchKernelGGL(k_col_partial, dim3(nb, ncol), dim3(LT), 0, st, R, ldr, T, ldt, cidx, h->dev->kappa, h->L,
                     *part);
  hipLaunchKernelGGL(k_col_finish, dim3((ncol + 63) / 64), dim3(64), 0, st, *part, nb, ncol, lam, cidx, *cols);
  HIP_TRY_L(hipGetLastError());
  *nb_out = nb;
  return HELIC_OK;
}

helic_status apply_impl(helic_basis_s* h, const helic_lpc_s* net, const double* R, int64_t ldr, const double* lam,
                        double* W, int64_t ldw, int nvec, hipStream_t st) {
  helic_status s = ready(h);
  if (s) return s;
  double* part;
  ColRec* cols;
  int nb;
  if ((s = column_records(h, R, ldr, nullptr, 0, nullptr, lam, nvec, st, &part, &cols, &nb))) return s;
  hipLaunchKernelGGL(k_lpc_apply, dim3(nb, nvec), dim3(LT), 0, st, R, ldr, W, ldw, h->dev->kappa, h->dev->vdiag,
                     h->L, std::sqrt((double)h->L), cols, net->theta);
  HIP_TRY_L(hipGetLastError());
  return HELIC_OK;
}

helic_status loss_grad_impl(helic_basis_s* h, helic_lpc_s* net, const double* R, int64_t ldr, const double* T,
                            int64_t ldt, const int32_t* cidx, const double* lam, int ncol, hipStream_t st,
                            double* loss) {
  helic_status s = ready(h);
  if (s) return s;
  double* part;
  ColRec* cols;
  int nb;
  if ((s = column_records(h, R, ldr, T, ldt, cidx, lam, ncol, st, &part, &cols, &nb))) return s;
  const double sqrtL = std::sqrt((double)h->L);
  hipLaunchKernelGGL(k_lpc_fwd_partial, dim3(nb, ncol), dim3(LT), 0, st, R, ldr, T, ldt, cidx, h->dev->kappa,
                     h->dev->vdiag, h->L, sqrtL, cols, net->theta, part);
  hipLaunchKernelGGL(k_loss_finish, dim3((ncol + 63) / 64), dim3(64), 0, st, part, nb, ncol, cols);
  HIP_TRY_L(hipGetLastError());
  const int64_t ntiles = (h->L * ncol + LT - 1) / LT;
  int ncu = 256;
  {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, net->device) == hipSuccess && pr.multiProcessorCount > 0)
      ncu = pr.multiProcessorCount;
  }
  const int nwg = (int)std::min<int64_t>(ntiles, 2 * ncu);
  const size_t need = (size_t)nwg * NPAD * sizeof(float);
  if (need > net->gpart_bytes) {
    if (net->gpart) HIP_TRY_L(hipFree(net->gpart));
    net->gpart = nullptr;
    net->gpart_bytes = 0;
    HIP_TRY_L(hipMalloc((void**)&net->gpart, need));
    net->gpart_bytes = need;
  }
  HIP_TRY_L(hipFuncSetAttribute((const void*)k_lpc_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)BWD_LDS));
  hipLaunchKernelGGL(k_lpc_backward, dim3(nwg), dim3(LT), BWD_LDS, st, R, ldr, T, ldt, cidx, h->dev->kappa,
                     h->dev->vdiag, h->L, ncol, sqrtL, cols, net->theta, net->gpart, ntiles);
  hipLaunchKernelGGL(k_grad_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, st, net->gpart, nwg, net->grad);
  HIP_TRY_L(hipGetLastError());
  if (loss) {
    std::vector<ColRec> hc(ncol);
    HIP_TRY_L(hipMemcpyAsync(hc.data(), cols, sizeof(ColRec) * ncol, hipMemcpyDeviceToHost, st));
    HIP_TRY_L(hipStreamSynchronize(st));
    double acc = 0.0;
    for (const ColRec& c : hc) acc += c.loss;
    *loss = acc / ncol;
  }
  return HELIC_OK;
}

helic_status adam_impl(helic_lpc_s* net, double lr, hipStream_t st) {
  ++net->step;
  const float bc1 = (float)(1.0 - std::pow(0.9, net->step)), bc2 = (float)(1.0 - std::pow(0.999, net->step));
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, net->theta, net->m, net->v, net->grad,
                     (float)lr, bc1, bc2);
  HIP_TRY_L(hipGetLastError());
  return HELIC_OK;
}

}  // namespace

// Solver hook: the attached network, else an error (the caller asked for it).
helic_status lpc_precondition(helic_basis_s* h, const double* Rr, int64_t ldr, const double* lam, double* W,
                              int64_t ldw, int nvec, hipStream_t st) {
  if (!h->dev || !h->dev->lpc) return fail(HELIC_ERR_STATE, "no learned preconditioner attached");
  return apply_impl(h, h->dev->lpc, Rr, ldr, lam, W, ldw, nvec, st);
}

bool lpc_attached(const helic_basis_s* h) { return h->dev && h->dev->lpc; }

}  // namespace helic

using namespace helic;

extern "C" {

helic_status helic_lpc_create(uint64_t seed, helic_lpc* out) {
  if (!out) return fail(HELIC_ERR_INVALID, "null argument");
  *out = nullptr;
  helic_lpc_s* net = new (std::nothrow) helic_lpc_s();
  if (!net) return fail(HELIC_ERR_NOMEM, "host allocation failed");
  auto bad = [&](hipError_t e) -> helic_status {
    helic_lpc_destroy(net);
    return fail(HELIC_ERR_HIP, std::string("network allocation: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&net->device)) != hipSuccess) return bad(e);
  if ((e = hipMalloc((void**)&net->theta, NPAD * sizeof(float))) != hipSuccess) return bad(e);
  if ((e = hipMalloc((void**)&net->m, NPAD * sizeof(float))) != hipSuccess) return bad(e);
  if ((e = hipMalloc((void**)&net->v, NPAD * sizeof(float))) != hipSuccess) return bad(e);
  if ((e = hipMalloc((void**)&net->grad, NPAD * sizeof(double))) != hipSuccess) return bad(e);
  std::vector<float> p(NPAD, 0.0f);
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int i = 0; i < HID * NIN; ++i) p[P_W1 + i] = (float)(nd(gen) * std::sqrt(2.0 / NIN));
  for (int i = 0; i < HID * HID; ++i) p[P_W2 + i] = (float)(nd(gen) * std::sqrt(2.0 / HID));
  helic_status s = helic_lpc_set_params(net, p.data());
  if (s) {
    helic_lpc_destroy(net);
    return s;
  }
  *out = net;
  return HELIC_OK;
}

helic_status helic_lpc_destroy(helic_lpc net) {
  if (!net) return HELIC_OK;
  void* ptrs[] = {net->theta, net->m, net->v, net->grad, net->gpart, net->tidx};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete net;
  return HELIC_OK;
}

helic_status helic_lpc_get_params(helic_lpc net, float* params) {
  if (!net || !params) return fail(HELIC_ERR_INVALID, "null argument");
  helic_status s = check_net(net);
  if (s) return s;
  HIP_TRY_L(hipMemcpy(params, net->theta, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  return HELIC_OK;
}

helic_status helic_lpc_set_params(helic_lpc net, const float* params) {
  if (!net || !params) return fail(HELIC_ERR_INVALID, "null argument");
  helic_status s = check_net(net);
  if (s) return s;
  for (int i = 0; i < NPARAM; ++i)
    if (!std::isfinite(params[i])) return fail(HELIC_ERR_INVALID, "non-finite parameter " + std::to_string(i));
  std::vector<float> p(NPAD, 0.0f);
  std::memcpy(p.data(), params, NPARAM * sizeof(float));
  HIP_TRY_L(hipMemcpy(net->theta, p.data(), NPAD * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY_L(hipMemset(net->m, 0, NPAD * sizeof(float)));
  HIP_TRY_L(hipMemset(net->v, 0, NPAD * sizeof(float)));
  HIP_TRY_L(hipMemset(net->grad, 0, NPAD * sizeof(double)));
  net->step = 0;
  return HELIC_OK;
}

helic_status helic_lpc_save(helic_lpc net, const char* path) {
  if (!net || !path) return fail(HELIC_ERR_INVALID, "null argument");
  std::vector<float> p(NPARAM);
  helic_status s = helic_lpc_get_params(net, p.data());
  if (s) return s;
  unsigned char head[16] = {'H', 'E', 'L', 'I', 'C', 'L', 'P', 'C'};
  const int32_t version = 1, count = NPARAM;
  for (int b = 0; b < 4; ++b) {
    head[8 + b] = (unsigned char)((version >> (8 * b)) & 0xff);
    head[12 + b] = (unsigned char)((count >> (8 * b)) & 0xff);
  }
  std::vector<unsigned char> body((size_t)NPARAM * 4);
  for (int i = 0; i < NPARAM; ++i) {
    uint32_t u;
    std::memcpy(&u, &p[i], 4);
    for (int b = 0; b < 4; ++b) body[(size_t)4 * i + b] = (unsigned char)((u >> (8 * b)) & 0xff);
  }
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(HELIC_ERR_INVALID, std::string("cannot open ") + path + " for writing");
  const bool ok = std::fwrite(head, 1, 16, f) == 16 && std::fwrite(body.data(), 1, body.size(), f) == body.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed) return fail(HELIC_ERR_INVALID, std::string("cannot write ") + path);
  return HELIC_OK;
}

helic_status helic_lpc_load(helic_lpc net, const char* path) {
  if (!net || !path) return fail(HELIC_ERR_INVALID, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(HELIC_ERR_INVALID, std::string("cannot open ") + path);
  unsigned char head[16];
  std::vector<unsigned char> body((size_t)NPARAM * 4 + 1);
  const size_t nh = std::fread(head, 1, 16, f);
  const size_t nb = nh == 16 ? std::fread(body.data(), 1, body.size(), f) : 0;
  std::fclose(f);
  auto le32 = [&](int o) {
    return (int32_t)((uint32_t)head[o] | ((uint32_t)head[o + 1] << 8) | ((uint32_t)head[o + 2] << 16) |
                     ((uint32_t)head[o + 3] << 24));
  };
  if (nh != 16 || std::memcmp(head, "HELICLPC", 8) != 0 || le32(8) != 1 || le32(12) != NPARAM ||
      nb != (size_t)NPARAM * 4)
    return fail(HELIC_ERR_INVALID, std::string(path) + " is not a weights file of this network");
  std::vector<float> p(NPARAM);
  for (int i = 0; i < NPARAM; ++i) {
    uint32_t u = 0;
    for (int b = 0; b < 4; ++b) u |= (uint32_t)body[(size_t)4 * i + b] << (8 * b);
    std::memcpy(&p[i], &u, 4);
  }
  return helic_lpc_set_params(net, p.data());
}

helic_status helic_lpc_attach(helic_basis h, helic_lpc net) {
  if (!h) return fail(HELIC_ERR_INVALID, "null argument");
  if (!h->dev) return fail(HELIC_ERR_STATE, "no potential set");
  if (net) {
    helic_status s = check_net(net);
    if (s) return s;
  }
  h->dev->lpc = net;
  return HELIC_OK;
}

helic_status helic_lpc_vdiag(helic_basis h, double* vdiag) {
  if (!h || !vdiag) return fail(HELIC_ERR_INVALID, "null argument");
  helic_status s = ready(h);
  if (s) return s;
  HIP_TRY_L(hipDeviceSynchronize());   // the potential may have been set on any stream
  HIP_TRY_L(hipMemcpy(vdiag, h->dev->vdiag, sizeof(double) * h->L, hipMemcpyDeviceToHost));
  return HELIC_OK;
}

helic_status helic_lpc_apply(helic_basis h, helic_lpc net, const double* R, int64_t ldr, const double* lam,
                             double* W, int64_t ldw, int32_t nvec, void* stream) {
  if (!h || !net || !R || !lam || !W) return fail(HELIC_ERR_INVALID, "null argument");
  if (nvec < 1 || ldr < h->L || ldw < h->L || nvec > 65535) return fail(HELIC_ERR_INVALID, "bad block shape");
  helic_status s = check_net(net);
  if (s) return s;
  return apply_impl(h, net, R, ldr, lam, W, ldw, nvec, reinterpret_cast<hipStream_t>(stream));
}

helic_status helic_lpc_loss_grad(helic_basis h, helic_lpc net, const double* R, int64_t ldr, const double* T,
                                 int64_t ldt, const double* lam, int32_t nvec, double* loss, double* grad,
                                 void* stream) {
  if (!h || !net || !R || !T || !lam || !loss) return fail(HELIC_ERR_INVALID, "null argument");
  if (nvec < 1 || ldr < h->L || ldt < h->L || nvec > 65535) return fail(HELIC_ERR_INVALID, "bad block shape");
  helic_status s = check_net(net);
  if (s) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((s = loss_grad_impl(h, net, R, ldr, T, ldt, nullptr, lam, nvec, st, loss))) return s;
  if (grad) {
    HIP_TRY_L(hipMemcpyAsync(grad, net->grad, sizeof(double) * NPARAM, hipMemcpyDeviceToHost, st));
    HIP_TRY_L(hipStreamSynchronize(st));
  }
  return HELIC_OK;
}

helic_status helic_lpc_adam_step(helic_lpc net, double lr, void* stream) {
  if (!net) return fail(HELIC_ERR_INVALID, "null argument");
  if (!(lr > 0.0)) return fail(HELIC_ERR_INVALID, "learning rate must be positive");
  helic_status s = check_net(net);
  if (s) return s;
  return adam_impl(net, lr, reinterpret_cast<hipStream_t>(stream));
}

helic_status helic_lpc_train(helic_basis h, helic_lpc net, const double* R, int64_t ldr, const double* T,
                             int64_t ldt, const double* lam, int32_t ncol, int32_t batch, int32_t steps,
                             double lr, uint64_t seed, double* losses, void* stream) {
  if (!h || !net || !R || !T || !lam) return fail(HELIC_ERR_INVALID, "null argument");
  if (ncol < 1 || batch < 1 || batch > ncol || steps < 0 || ldr < h->L || ldt < h->L || !(lr > 0.0))
    return fail(HELIC_ERR_INVALID, "bad training arguments");
  helic_status s = check_net(net);
  if (s) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (net->tidx_n < batch) {
    if (net->tidx) HIP_TRY_L(hipFree(net->tidx));
    net->tidx = nullptr;
    net->tidx_n = 0;
    HIP_TRY_L(hipMalloc((void**)&net->tidx, sizeof(int32_t) * batch));
    net->tidx_n = batch;
  }
  std::mt19937_64 gen(seed);
  std::vector<int32_t> perm(ncol);
  for (int i = 0; i < ncol; ++i) perm[i] = i;
  std::vector<int32_t> pick(batch);
  for (int it = 0; it < steps; ++it) {
    for (int q = 0; q < batch; ++q) {   // partial Fisher-Yates: a uniform sample without replacement
      std::uniform_int_distribution<int> u(q, ncol - 1);
      std::swap(perm[q], perm[u(gen)]);
      pick[q] = perm[q];
    }
    std::sort(pick.begin(), pick.end());
    HIP_TRY_L(hipMemcpyAsync(net->tidx, pick.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice, st));
    double loss = 0.0;   // reading the loss also orders the next index upload after this step
    if ((s = loss_grad_impl(h, net, R, ldr, T, ldt, net->tidx, lam, batch, st, &loss))) return s;
    if ((s = adam_impl(net, lr, st))) return s;
    if (losses) losses[it] = loss;
  }
  HIP_TRY_L(hipStreamSynchronize(st));
  return HELIC_OK;
}

}  // extern "C"
