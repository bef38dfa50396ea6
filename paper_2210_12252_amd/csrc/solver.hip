// Block eigensolver for the lowest eigenpairs of H: LOBPCG (Sec. 3.5) with
// soft locking and the Teter-Payne-Allan preconditioner.  Each iteration
// forms the trial space S = [X, W, P] (Ritz vectors, preconditioned
// residuals, previous update directions); W is projected against X and P
// against [X, W] (twice each) and both are orthonormalised (Cholesky QR
// twice, SVQB if rank deficient), so S is orthonormal and the FP64
// Rayleigh-Ritz step is the Hermitian eigenproblem of S^H (H S) (ZGEMM by
// rocBLAS, eigen-decomposition by rocSOLVER).  With FP32 H*X the iteration
// locks columns at switch_tol until every wanted residual is below it,
// recomputes H X and H P in FP64 and continues in FP64 to tol.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "device_state.hpp"
#include "helic_internal.h"

namespace helic {

helic_status apply_H_impl(helic_basis_s* h, const double* X, int64_t ldx, double* Y, int64_t ldy, int nvec,
                          helic_prec prec, hipStream_t st, int chunk);
helic_status ensure_workspace(helic_basis_s* h, int nvec, size_t elem);
size_t slab_elem_bytes(helic_prec prec);
helic_status precondition_impl(helic_basis_s* h, const double* Rr, int64_t ldr, double* W, int64_t ldw,
                               int nvec, hipStream_t st);
helic_status lpc_precondition(helic_basis_s* h, const double* Rr, int64_t ldr, const double* lam, double* W,
                              int64_t ldw, int nvec, hipStream_t st);
bool lpc_attached(const helic_basis_s* h);

// Training pairs for the learned preconditioner taken during a solve: at the
// scheduled iterations the residuals of the unconverged wanted columns (and
// the Ritz block) are kept; targets are formed after convergence.
struct Harvest {
  int n_snap = 0, max_cols = 0;
  double *R = nullptr, *T = nullptr, *lam = nullptr;   // outputs (device, ld = L)
  int ncol = 0;
  int next_iter = 0;                  // next scheduled iteration
  struct Snap {
    int col0, ncols;
    double* X;                        // Ritz block at the snapshot (n columns)
    std::vector<int32_t> ritz;        // Ritz index of each kept column
  };
  std::vector<Snap> snaps;
  std::vector<double> lam_h;
  ~Harvest() {
    for (Snap& s : snaps)
      if (s.X) (void)hipFree(s.X);
  }
};

void release_solver_state(DeviceState*) {}

namespace {

typedef rocblas_double_complex zc;
constexpr int NTS = 256;

#define HIP_TRY_S(call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(HELIC_ERR_HIP, std::string(#call) + " (solver line " + std::to_string(__LINE__) + "): " + \
                                     hipGetErrorString(e_));                          \
  } while (0)
#define RB_TRY(call)                                                                  \
  do {                                                                                \
    rocblas_status e_ = (call);                                                       \
    if (e_ != rocblas_status_success)                                                 \
      return fail(HELIC_ERR_HIP, std::string(#call) + ": rocblas status " +          \
                                     std::to_string((int)e_));                        \
  } while (0)

// R_j = AX_j - lam_j X_j and partial sums of |R_j|^2 over row chunks
__global__ void __launch_bounds__(NTS)
k_residual(const double* __restrict__ AX, const double* __restrict__ X, const double* __restrict__ lam,
           double* __restrict__ R, int64_t L, int nchunk, double* __restrict__ part) {
  __shared__ double red[NTS];
  const int c = blockIdx.x, j = blockIdx.y;
  const int64_t per = (L + nchunk - 1) / nchunk;
  const int64_t lo = c * per, hi = std::min(L, lo + per);
  const double l = lam[j];
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += NTS) {
    const int64_t o = ((int64_t)j * L + i) * 2;
    const double re = AX[o] - l * X[o], im = AX[o + 1] - l * X[o + 1];
    R[o] = re;
    R[o + 1] = im;
    s += re * re + im * im;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NTS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)j * nchunk + c] = red[0];
}

__global__ void k_finish_norms(const double* __restrict__ part, int nchunk, int ncol, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)j * nchunk + c];
  out[j] = std::sqrt(s);
}

// dst[:, c] = src[:, idx[c]] for c < ncol (columns of length L complex)
__global__ void __launch_bounds__(NTS)
k_gather_cols(const double* __restrict__ src, double* __restrict__ dst, const int32_t* __restrict__ idx,
              int64_t L, int ncol) {
  const int c = blockIdx.y;
  if (c >= ncol) return;
  const double* s = src + (int64_t)idx[c] * L * 2;
  double* d = dst + (int64_t)c * L * 2;
  for (int64_t i = blockIdx.x * (int64_t)NTS + threadIdx.x; i < 2 * L; i += (int64_t)gridDim.x * NTS) d[i] = s[i];
}

// d_i = 1 / sqrt(Re G_ii) (0 if not positive); G_ij <- d_i d_j G_ij
__global__ void k_svqb_scale(double* __restrict__ G, int k, int ld, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    const double g = G[((int64_t)i * ld + i) * 2];
    d[i] = g > 0.0 ? 1.0 / std::sqrt(g) : 0.0;
  }
}
__global__ void k_scale_sym(double* __restrict__ G, int k, int ld, const double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < k && j < k) {
    const double s = d[i] * d[j];
    G[((int64_t)j * ld + i) * 2] *= s;
    G[((int64_t)j * ld + i) * 2 + 1] *= s;
  }
}
// Z[:, c] = D U[:, i0 + c] / sqrt(theta[i0 + c]), c < kk
__global__ void k_make_Z(const double* __restrict__ U, int ldu, const double* __restrict__ d,
                         const double* __restrict__ theta, int i0, int k, int kk, double* __restrict__ Z, int ldz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (i < k && c < kk) {
    const double s = d[i] / std::sqrt(theta[i0 + c]);
    Z[((int64_t)c * ldz + i) * 2] = U[((int64_t)(i0 + c) * ldu + i) * 2] * s;
    Z[((int64_t)c * ldz + i) * 2 + 1] = U[((int64_t)(i0 + c) * ldu + i) * 2 + 1] * s;
  }
}

// T[c * ldt + r] = C[(idx[c]) * ldc + r0 + r], r < nr, c < nc (complex)
__global__ void k_gather_sub(const double* __restrict__ Cm, int ldc, int r0, int nr, const int32_t* __restrict__ idx,
                             int nc, double* __restrict__ T, int ldt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r < nr && c < nc) {
    const int64_t so = ((int64_t)idx[c] * ldc + r0 + r) * 2, dO = ((int64_t)c * ldt + r) * 2;
    T[dO] = Cm[so];
    T[dO + 1] = Cm[so + 1];
  }
}

// C[i + j ldc] = beta C + sum_b P[b][i + j m] (complex), the split-K partials
__global__ void k_reduce_partials(const double* __restrict__ P, int nb, int m, int nn, double* __restrict__ Cm,
                                  int ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= m || j >= nn) return;
  double re = 0.0, im = 0.0;
  const size_t stride = (size_t)m * nn * 2;
  for (int b = 0; b < nb; ++b) {
    re += P[b * stride + ((size_t)j * m + i) * 2];
    im += P[b * stride + ((size_t)j * m + i) * 2 + 1];
  }
  Cm[((size_t)j * ldc + i) * 2] = re;
  Cm[((size_t)j * ldc + i) * 2 + 1] = im;
}

// Standard normal numbers from a counter-based generator, the same for any
// launch shape: the SplitMix64 finaliser (Steele, Lea and Flood 2014) of the
// seed and the element index gives two 53-bit uniforms, and the Box-Muller
// transform maps them to one normal.
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(NTS) k_random_normal(double* __restrict__ out, int64_t n, uint64_t seed) {
  const uint64_t key = mix64(seed);
  for (int64_t i = blockIdx.x * (int64_t)NTS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTS) {
    const uint64_t a = mix64(key ^ (2 * (uint64_t)i)), b = mix64(key ^ (2 * (uint64_t)i + 1));
    const double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;   // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1.0p-53;         // [0, 1)
    out[i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
  }
}

// C[0:m, 0:m] (ld ldc, complex) = diag(lam)
__global__ void k_diag_block(double* __restrict__ Cm, int ldc, const double* __restrict__ lam, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= m) return;
  Cm[((size_t)j * ldc + i) * 2] = i == j ? lam[i] : 0.0;
  Cm[((size_t)j * ldc + i) * 2 + 1] = 0.0;
}

// One step of the scaled Chebyshev recurrence, elementwise over n doubles:
// Out = alpha (AY - c Y) + beta Xp (Xp is not read when beta = 0).  Out may
// be Xp: each element is read before it is written, by the same thread.
__global__ void __launch_bounds__(NTS)
k_cheb_step(const double* __restrict__ AY, const double* __restrict__ Y, const double* Xp, double* Out, int64_t n,
            double alpha, double c, double beta) {
  for (int64_t i = blockIdx.x * (int64_t)NTS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTS) {
    const double f = alpha * (AY[i] - c * Y[i]);
    Out[i] = beta != 0.0 ? f + beta * Xp[i] : f;
  }
}

// The same step with its coefficients (alpha, c, beta) read from device
// memory, so that a captured graph of the recurrence replays with the
// coefficients of each outer step.
__global__ void __launch_bounds__(NTS)
k_cheb_step_c(const double* __restrict__ AY, const double* __restrict__ Y, const double* Xp, double* Out, int64_t n,
              const double* __restrict__ coef) {
  const double alpha = coef[0], c = coef[1], beta = coef[2];
  for (int64_t i = blockIdx.x * (int64_t)NTS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTS) {
    const double f = alpha * (AY[i] - c * Y[i]);
    Out[i] = beta != 0.0 ? f + beta * Xp[i] : f;
  }
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal d and off-diagonal e (Sturm sequence of the LDL^T pivots).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Largest eigenvalue of that matrix by bisection inside its Gershgorin interval.
double tridiag_max_eig(const std::vector<double>& d, const std::vector<double>& e) {
  double lo = HUGE_VAL, hi = -HUGE_VAL;
  for (size_t i = 0; i < d.size(); ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < d.size() ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  const int n = (int)d.size();
  for (int k = 0; k < 200 && hi - lo > 1e-14 * std::max(1.0, std::fabs(hi)); ++k) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, mid) >= n) hi = mid; else lo = mid;
  }
  return hi;
}

struct Bufs {
  std::vector<void*> owned;
  ~Bufs() {
    for (void* p : owned) (void)hipFree(p);
  }
  helic_status get(double** p, size_t n) {
    HIP_TRY_S(hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(double)));
    owned.push_back(*p);
    return HELIC_OK;
  }
};

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

}  // namespace

helic_status eigensolve_impl(helic_basis_s* h, const helic_solve_opts& o, double* evals, double* resid,
                             double* evecs, int64_t ldv, helic_solve_stats* stats, hipStream_t st, Harvest* hv,
                             int cheb_degree, bool allow_graph) {
  Timer total;
  helic_solve_stats S_;
  std::memset(&S_, 0, sizeof(S_));
  const int64_t L = h->L;
  // The solve runs on a stream of its own when the caller passes the null
  // stream (which cannot be captured into a graph); the caller's earlier work
  // is waited for first, and everything is synchronised before returning.
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    }
  } own;
  if (!st) {
    HIP_TRY_S(hipStreamSynchronize(nullptr));
    HIP_TRY_S(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking));
    st = own.s;
  }
  const int nev = o.nev;
  // automatic guard: a wider block speeds the filter's convergence (the
  // damped interval starts further above the wanted eigenvalues)
  const int guard = o.guard >= 0 ? o.guard : cheb_degree > 0 ? std::max(8, nev / 3) : std::max(4, nev / 8);
  const int n = (int)std::min<int64_t>(L, (int64_t)nev + guard);
  const int chunk = std::max(1, std::min(o.block, 64));
  const int kmax = 3 * n;
  helic_prec prec = (helic_prec)o.prec;
  const double switch_tol = o.switch_tol > 0 ? o.switch_tol : 1e-5;
  // BF16 start: FP32 takes over below switch_bf16, FP64 below switch_tol
  const double switch_bf16 = std::max(switch_tol, o.switch_tol_bf16 > 0 ? o.switch_tol_bf16 : 1e-2);
  // A low-precision phase also ends when its worst wanted residual has not
  // improved by 10 % for this many iterations (filter steps): below the
  // precision's own error floor its switch tolerance may be out of reach.
  const int stall_limit = cheb_degree > 0 ? 3 : 10;
  double phase_best = HUGE_VAL;
  int phase_stall = 0;
  auto stalled = [&](double worst) {
    if (prec == HELIC_FP64) return false;
    if (worst < 0.9 * phase_best) {
      phase_best = worst;
      phase_stall = 0;
    } else {
      ++phase_stall;
    }
    return phase_stall >= stall_limit;
  };
  auto prec_name = [&]() { return prec == HELIC_FP64 ? "FP64" : prec == HELIC_FP32 ? "FP32" : "BF16"; };
  // lock tolerance of the low-precision phases: where their H*X stops improving a column
  auto phase_tol = [&]() { return prec == HELIC_FP64 ? o.tol : std::max(o.tol, prec == HELIC_FP32 ? switch_tol : switch_bf16); };
  bool stopped_low = false;   // o.stop_low: ended at the first precision switch

  Bufs B;
  double *S, *AS, *Pb, *APb, *Xn, *AXn, *R, *GA, *Z, *T1, *C, *theta, *E, *d, *lam, *part, *norms, *jres;
  const size_t Lc = (size_t)L * 2;   // doubles per complex column
  const size_t KK = (size_t)kmax * kmax * 2;
  helic_status s;
  if ((s = B.get(&S, Lc * kmax)) || (s = B.get(&AS, Lc * kmax)) || (s = B.get(&Pb, Lc * n)) ||
      (s = B.get(&APb, Lc * n)) || (s = B.get(&Xn, Lc * n)) || (s = B.get(&AXn, Lc * n)) ||
      (s = B.get(&R, Lc * n)) || (s = B.get(&GA, KK)) || (s = B.get(&Z, KK)) || (s = B.get(&T1, KK)) ||
      (s = B.get(&C, KK)) || (s = B.get(&theta, kmax)) || (s = B.get(&E, kmax)) || (s = B.get(&d, kmax)) ||
      (s = B.get(&lam, kmax)) || (s = B.get(&norms, kmax)) || (s = B.get(&jres, 1)))
    return s;
  const int nchunk = (int)std::min<int64_t>(64, (L + 2047) / 2048);
  if ((s = B.get(&part, (size_t)nchunk * n))) return s;
  // split-K Gram products: the long row dimension L is cut into nsplit slices
  // (one batched ZGEMM), partial k x k results are summed by a small kernel
  const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(32, L / 1024));
  const int64_t slice = L / nsplit;   // the last slice also takes L - nsplit * slice rows
  double* gpart = nullptr;
  if ((s = B.get(&gpart, (size_t)(nsplit + 1) * kmax * kmax * 2))) return s;
  double* lz = nullptr;   // Lanczos columns of the Chebyshev-filtered solver
  if (cheb_degree > 0 && (s = B.get(&lz, Lc * 3))) return s;
  int32_t *d_idx = nullptr, *d_info = nullptr, *d_sweeps = nullptr;
  HIP_TRY_S(hipMalloc((void**)&d_idx, sizeof(int32_t) * n));
  B.owned.push_back(d_idx);
  HIP_TRY_S(hipMalloc((void**)&d_info, sizeof(int32_t)));
  B.owned.push_back(d_info);
  HIP_TRY_S(hipMalloc((void**)&d_sweeps, sizeof(int32_t)));
  B.owned.push_back(d_sweeps);

  rocblas_handle rb = nullptr;
  RB_TRY(rocblas_create_handle(&rb));
  struct HandleGuard {
    rocblas_handle h;
    ~HandleGuard() { rocblas_destroy_handle(h); }
  } hg{rb};
  RB_TRY(rocblas_set_stream(rb, st));
  const zc one{1.0, 0.0}, zero{0.0, 0.0}, mone{-1.0, 0.0};
  auto col = [&](double* base, int c) { return base + (size_t)c * Lc; };
  auto sync = [&]() -> helic_status {
    HIP_TRY_S(hipStreamSynchronize(st));
    return HELIC_OK;
  };

  // Cm (m x nn, ld ldc) = A^H Bm for L-row blocks A (m columns) and Bm (nn columns)
  auto gemm_h = [&](int m, int nn, const double* A, const double* Bm, double* Cm, int ldc) -> helic_status {
    if (m == 0 || nn == 0) return HELIC_OK;
    RB_TRY(rocblas_zgemm_strided_batched(rb, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, nn,
                                         (int)slice, &one, (const zc*)A, (int)L, slice, (const zc*)Bm, (int)L, slice,
                                         &zero, (zc*)gpart, m, (int64_t)m * nn, nsplit));
    int nb = nsplit;
    const int64_t rem = L - (int64_t)nsplit * slice;
    if (rem > 0) {
      const size_t off = (size_t)nsplit * slice * 2;
      RB_TRY(rocblas_zgemm(rb, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, nn, (int)rem, &one,
                           (const zc*)(A + off), (int)L, (const zc*)(Bm + off), (int)L, &zero,
                           (zc*)(gpart + (size_t)nsplit * m * nn * 2), m));
      ++nb;
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3((m + 63) / 64, nn), dim3(64), 0, st, gpart, nb, m, nn, Cm, ldc);
    HIP_TRY_S(hipGetLastError());
    return HELIC_OK;
  };

  auto apply = [&](const double* X, double* Y, int nv) -> helic_status {
    if (nv == 0) return HELIC_OK;
    Timer t;
    helic_status r = apply_H_impl(h, X, L, Y, L, nv, prec, st, chunk);
    if (r != HELIC_OK) return r;
    HIP_TRY_S(hipStreamSynchronize(st));
    S_.t_apply_ms += t.ms();
    S_.n_apply += nv;
    return HELIC_OK;
  };

  // Hermitian eigen-decomposition of the k x k matrix A (ld kmax) in place,
  // eigenvalues ascending in w (device) and wh (host).  Divide and conquer
  // first; it returns NaN on exactly deflating (identity-block) matrices of
  // order >= 90, so a non-finite or failed result is redone by Jacobi from a
  // copy of the input.
  auto heev = [&](int k, double* A, double* w, std::vector<double>& wh) -> helic_status {
    const size_t bytes = (size_t)kmax * k * 2 * sizeof(double);
    HIP_TRY_S(hipMemcpyAsync(Z, A, bytes, hipMemcpyDeviceToDevice, st));
    RB_TRY(rocsolver_zheevd(rb, rocblas_evect_original, rocblas_fill_upper, k, (zc*)A, kmax, w, E, d_info));
    wh.resize(k);
    int32_t info = 0;
    HIP_TRY_S(hipMemcpyAsync(wh.data(), w, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIP_TRY_S(hipMemcpyAsync(&info, d_info, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY_S(hipStreamSynchronize(st));
    bool ok = info == 0;
    for (int i = 0; i < k && ok; ++i) ok = std::isfinite(wh[i]);
    if (ok) return HELIC_OK;
    HIP_TRY_S(hipMemcpyAsync(A, Z, bytes, hipMemcpyDeviceToDevice, st));
    RB_TRY(rocsolver_zheevj(rb, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper, k, (zc*)A,
                            kmax, 0.0, jres, 100, d_sweeps, w, d_info));
    HIP_TRY_S(hipMemcpyAsync(wh.data(), w, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIP_TRY_S(hipMemcpyAsync(&info, d_info, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY_S(hipStreamSynchronize(st));
    ok = info == 0;
    for (int i = 0; i < k && ok; ++i) ok = std::isfinite(wh[i]);
    if (!ok) return fail(HELIC_ERR_NOCONV, "small Hermitian eigenproblem failed");
    return HELIC_OK;
  };

  // Orthonormalise the ncols columns at Y (same transform on AY when given):
  // Cholesky QR twice; if the Gram matrix is not numerically positive
  // definite, SVQB (scaled Gram eigen-decomposition, directions below 1e-12
  // of the largest dropped).  *kept receives the new column count.
  auto ortho_block = [&](double* Y, double* AY, int ncols, int* kept) -> helic_status {
    bool svqb_done = false;
    for (int pass = 0; pass < 2 && ncols > 0; ++pass) {
      if ((s = gemm_h(ncols, ncols, Y, Y, T1, kmax))) return s;
      HIP_TRY_S(hipMemcpyAsync(GA, T1, (size_t)kmax * ncols * 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
      RB_TRY(rocsolver_zpotrf(rb, rocblas_fill_upper, ncols, (zc*)T1, kmax, d_info));
      int32_t info = 0;
      HIP_TRY_S(hipMemcpyAsync(&info, d_info, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY_S(hipStreamSynchronize(st));
      if (info == 0) {
        RB_TRY(rocblas_ztrsm(rb, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                             rocblas_diagonal_non_unit, (int)L, ncols, &one, (const zc*)T1, kmax, (zc*)Y, (int)L));
        if (AY)
          RB_TRY(rocblas_ztrsm(rb, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                               rocblas_diagonal_non_unit, (int)L, ncols, &one, (const zc*)T1, kmax, (zc*)AY, (int)L));
        continue;
      }
      if (svqb_done) return fail(HELIC_ERR_NOCONV, "block orthonormalisation failed");
      // SVQB on the saved Gram matrix, then the two Cholesky passes again
      hipLaunchKernelGGL(k_svqb_scale, dim3((ncols + 63) / 64), dim3(64), 0, st, GA, ncols, kmax, d);
      hipLaunchKernelGGL(k_scale_sym, dim3((ncols + 63) / 64, ncols), dim3(64), 0, st, GA, ncols, kmax, d);
      HIP_TRY_S(hipGetLastError());
      std::vector<double> th;
      if ((s = heev(ncols, GA, theta, th))) return s;
      const double tmax = th[ncols - 1];
      svqb_done = true;
      if (!(tmax > 0)) {
        ncols = 0;
        break;
      }
      int i0 = 0;
      while (i0 < ncols && th[i0] <= 1e-12 * tmax) ++i0;
      const int kk = ncols - i0;
      hipLaunchKernelGGL(k_make_Z, dim3((ncols + 63) / 64, kk), dim3(64), 0, st, GA, kmax, d, theta, i0, ncols, kk,
                         Z, kmax);
      HIP_TRY_S(hipGetLastError());
      RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, kk, ncols, &one, (const zc*)Y,
                           (int)L, (const zc*)Z, kmax, &zero, (zc*)Xn, (int)L));
      HIP_TRY_S(hipMemcpyAsync(Y, Xn, sizeof(double) * Lc * kk, hipMemcpyDeviceToDevice, st));
      if (AY) {
        RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, kk, ncols, &one,
                             (const zc*)AY, (int)L, (const zc*)Z, kmax, &zero, (zc*)AXn, (int)L));
        HIP_TRY_S(hipMemcpyAsync(AY, AXn, sizeof(double) * Lc * kk, hipMemcpyDeviceToDevice, st));
      }
      ncols = kk;
      pass = -1;
    }
    *kept = ncols;
    return HELIC_OK;
  };

  // Y -= B (B^H Y) and AY -= AB (B^H Y) for an orthonormal block B (nb columns)
  auto project = [&](const double* Bm, const double* ABm, int nb, double* Y, double* AY, int ny) -> helic_status {
    if (nb == 0 || ny == 0) return HELIC_OK;
    if ((s = gemm_h(nb, ny, Bm, Y, T1, kmax))) return s;
    RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, ny, nb, &mone, (const zc*)Bm,
                         (int)L, (const zc*)T1, kmax, &one, (zc*)Y, (int)L));
    if (AY)
      RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, ny, nb, &mone, (const zc*)ABm,
                           (int)L, (const zc*)T1, kmax, &one, (zc*)AY, (int)L));
    return HELIC_OK;
  };

  // Rayleigh-Ritz on the orthonormal S[:, base:base+k]: C = lowest `nout`
  // eigenvectors of S'^H (H S'), their eigenvalues into lam[base:] (device)
  // and lam_h[base:] (host); then X' <- S' C, AX' <- AS' C (in Xn/AXn from
  // column base).
  std::vector<double> lam_h(n, 0.0);
  auto rayleigh_ritz = [&](int base, int k, int nout, int nknown) -> helic_status {
    Timer t;
    // The leading nknown columns of S' are Ritz vectors with H X consistent,
    // so that block of S'^H (H S') is diag(lam); the eigensolver reads the
    // upper triangle only, so the Gram product needs columns nknown.. only.
    if (nknown > 0) {
      hipLaunchKernelGGL(k_diag_block, dim3((nknown + 63) / 64, nknown), dim3(64), 0, st, C, kmax, lam + base,
                         nknown);
      HIP_TRY_S(hipGetLastError());
    }
    if ((s = gemm_h(k, k - nknown, col(S, base), col(AS, base + nknown), C + (size_t)nknown * kmax * 2, kmax)))
      return s;
    std::vector<double> wh;
    if ((s = heev(k, C, lam + base, wh))) return s;
    for (int i = 0; i < nout; ++i) lam_h[base + i] = wh[i];
    RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, nout, k, &one,
                         (const zc*)col(S, base), (int)L, (const zc*)C, kmax, &zero, (zc*)col(Xn, base), (int)L));
    RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, nout, k, &one,
                         (const zc*)col(AS, base), (int)L, (const zc*)C, kmax, &zero, (zc*)col(AXn, base), (int)L));
    if ((s = sync())) return s;
    S_.t_rr_ms += t.ms();
    return HELIC_OK;
  };

  auto residuals = [&](std::vector<double>& nrm) -> helic_status {
    Timer t;
    hipLaunchKernelGGL(k_residual, dim3(nchunk, n), dim3(NTS), 0, st, AS, S, lam, R, L, nchunk, part);
    hipLaunchKernelGGL(k_finish_norms, dim3((n + 63) / 64), dim3(64), 0, st, part, nchunk, n, norms);
    HIP_TRY_S(hipGetLastError());
    nrm.resize(n);
    HIP_TRY_S(hipMemcpyAsync(nrm.data(), norms, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIP_TRY_S(hipStreamSynchronize(st));
    S_.t_precond_ms += t.ms();
    return HELIC_OK;
  };

  // Harvest: keep the residuals of the unconverged wanted columns (a prefix
  // of the ascending active list, gathered at W) and the Ritz block; the
  // next snapshot is due about 1.5 times later.
  auto snapshot = [&](int itn, const std::vector<int32_t>& act, const double* Wres, int na_) -> helic_status {
    hv->next_iter = std::max(itn + 1, (3 * itn) / 2);
    int m = 0;
    while (m < na_ && act[m] < nev) ++m;
    m = std::min(m, hv->max_cols - hv->ncol);
    if (m <= 0) return HELIC_OK;
    hv->snaps.push_back(Harvest::Snap{hv->ncol, m, nullptr, {}});
    Harvest::Snap& sp = hv->snaps.back();
    HIP_TRY_S(hipMalloc((void**)&sp.X, sizeof(double) * Lc * n));
    HIP_TRY_S(hipMemcpyAsync(sp.X, S, sizeof(double) * Lc * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY_S(hipMemcpyAsync(hv->R + (size_t)hv->ncol * Lc, Wres, sizeof(double) * Lc * m,
                             hipMemcpyDeviceToDevice, st));
    for (int c = 0; c < m; ++c) {
      sp.ritz.push_back(act[c]);
      hv->lam_h.push_back(lam_h[act[c]]);
    }
    hv->ncol += m;
    return HELIC_OK;
  };

  // Harvest targets T = (1 - Xs Xs^H) X* X*^H x for each kept column x of a
  // snapshot Xs, X* the converged wanted block (projection applied twice).
  auto harvest_targets = [&]() -> helic_status {
    for (const Harvest::Snap& sp : hv->snaps) {
      const int m = sp.ncols;
      double* T = hv->T + (size_t)sp.col0 * Lc;
      HIP_TRY_S(hipMemcpyAsync(d_idx, sp.ritz.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_gather_cols, dim3(64, m), dim3(NTS), 0, st, sp.X, R, d_idx, L, m);
      HIP_TRY_S(hipGetLastError());
      if ((s = gemm_h(nev, m, S, R, GA, kmax))) return s;
      RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, m, nev, &one,
                           (const zc*)S, (int)L, (const zc*)GA, kmax, &zero, (zc*)T, (int)L));
      for (int rep = 0; rep < 2; ++rep) {
        if ((s = gemm_h(n, m, sp.X, T, Z, kmax))) return s;
        RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, m, n, &mone,
                             (const zc*)sp.X, (int)L, (const zc*)Z, kmax, &one, (zc*)T, (int)L));
      }
      if ((s = sync())) return s;   // d_idx is reused by the next snapshot
    }
    if (hv->ncol > 0) {
      HIP_TRY_S(hipMemcpyAsync(hv->lam, hv->lam_h.data(), sizeof(double) * hv->ncol, hipMemcpyHostToDevice, st));
      if ((s = sync())) return s;
    }
    return HELIC_OK;
  };

  // ---- random start: orthonormalise, H X, first Rayleigh-Ritz
  {
    const int64_t nn = (int64_t)Lc * n;
    hipLaunchKernelGGL(k_random_normal, dim3((int)std::min<int64_t>(4096, (nn + NTS - 1) / NTS)), dim3(NTS), 0, st,
                       S, nn, o.seed);
    HIP_TRY_S(hipGetLastError());
    int kept = 0;
    if ((s = ortho_block(S, nullptr, n, &kept))) return s;
    if (kept < n) return fail(HELIC_ERR_NOCONV, "random start is rank deficient");
  }
  if ((s = apply(S, AS, n))) return s;
  if ((s = rayleigh_ritz(0, n, n, 0))) return s;
  HIP_TRY_S(hipMemcpyAsync(S, Xn, sizeof(double) * Lc * n, hipMemcpyDeviceToDevice, st));
  HIP_TRY_S(hipMemcpyAsync(AS, AXn, sizeof(double) * Lc * n, hipMemcpyDeviceToDevice, st));

  int np = 0;   // columns held in Pb / APb
  // learned preconditioner: dropped for the rest of the solve once the worst
  // wanted residual has not reached a new minimum for three iterations
  bool learned = o.precond == 2;
  double best_worst = HUGE_VAL;
  int stall = 0;
  std::vector<double> nrm;
  std::vector<int32_t> active, rel;
  // hard locking (FP64 phase): the leading nl columns, converged to tol, are
  // frozen; they stay in the projections of W and P but leave the
  // Rayleigh-Ritz problem, which shrinks to the other columns
  int nl = 0;
  bool exact_x = true;   // X^H (H X) = diag(lam) for the current Ritz block
  auto lowest_order = [&]() {   // columns by ascending Ritz value
    std::vector<int> ord(n);
    for (int j = 0; j < n; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return lam_h[a] < lam_h[b]; });
    return ord;
  };
  bool converged = false;
  int it = 0;
  if (cheb_degree > 0) {
    // ---- Chebyshev-filtered subspace iteration: per outer step the block
    // is filtered by a degree-m Chebyshev polynomial of H that damps the
    // interval [a, b] (a = the block's largest Ritz value, b = an upper bound
    // of the spectrum) and grows what lies below a, then orthonormalised and
    // rotated by FP64 Rayleigh-Ritz.  Scaled three-term recurrence (Zhou and
    // Saad, 2007), applied to the columns not yet locked.
    const int m = cheb_degree;
    std::vector<double> cheb_h(3 * (size_t)m);
    double* cheb_d = nullptr;
    if ((s = B.get(&cheb_d, 3 * (size_t)m))) return s;
    // captured filter recurrence (HELIC_CHEB_GRAPH=0 keeps eager launches).
    // Not for the concurrent solves of a batch: a capture in one host thread
    // makes the null-stream work that other threads' library set-up does
    // (rocBLAS / hipBLASLt initialisation, synchronous copies) fail with
    // hipErrorStreamCaptureImplicit.
    const char* ge = std::getenv("HELIC_CHEB_GRAPH");
    const bool use_graph = allow_graph && !(ge && ge[0] == '0');
    struct FilterGraph {
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      int nl = -1;
      helic_prec prec = HELIC_FP64;
      void reset() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        x = nullptr;
        g = nullptr;
        nl = -1;
      }
      ~FilterGraph() { reset(); }
    } fgraph;
    double b_up = 0.0;
    {
      // K-step Lanczos from one random column in FP64: the largest Ritz
      // value plus the last off-diagonal bounds the spectrum from above
      // (Zhou and Li, 2011)
      const int K = (int)std::min<int64_t>(12, L);
      double *v = lz, *vp = lz + Lc, *w = lz + 2 * Lc;
      hipLaunchKernelGGL(k_random_normal, dim3(64), dim3(NTS), 0, st, v, (int64_t)Lc, o.seed ^ 0x243f6a8885a308d3ull);
      HIP_TRY_S(hipGetLastError());
      double nv = 0.0;
      RB_TRY(rocblas_dznrm2(rb, (int)L, (const zc*)v, 1, &nv));
      if (!(nv > 0.0)) return fail(HELIC_ERR_NOCONV, "Lanczos start vector vanished");
      double inv = 1.0 / nv;
      RB_TRY(rocblas_zdscal(rb, (int)L, &inv, (zc*)v, 1));
      std::vector<double> al, be;
      for (int j = 0; j < K; ++j) {
        Timer t;
        if ((s = apply_H_impl(h, v, L, w, L, 1, HELIC_FP64, st, chunk))) return s;
        S_.n_apply += 1;
        zc dot;
        RB_TRY(rocblas_zdotc(rb, (int)L, (const zc*)v, 1, (const zc*)w, 1, &dot));
        S_.t_apply_ms += t.ms();
        const double a = reinterpret_cast<const double*>(&dot)[0];
        const zc ma{-a, 0.0};
        RB_TRY(rocblas_zaxpy(rb, (int)L, &ma, (const zc*)v, 1, (zc*)w, 1));
        if (j > 0) {
          const zc mb{-be.back(), 0.0};
          RB_TRY(rocblas_zaxpy(rb, (int)L, &mb, (const zc*)vp, 1, (zc*)w, 1));
        }
        double bn = 0.0;
        RB_TRY(rocblas_dznrm2(rb, (int)L, (const zc*)w, 1, &bn));
        al.push_back(a);
        be.push_back(bn);
        if (!(bn > 1e-12 * std::max(1.0, std::fabs(a)))) break;   // invariant subspace found
        double* t0 = vp;
        vp = v;
        v = w;
        w = t0;
        double ib = 1.0 / bn;
        RB_TRY(rocblas_zdscal(rb, (int)L, &ib, (zc*)v, 1));
      }
      const std::vector<double> off(be.begin(), be.end() - 1);
      b_up = tridiag_max_eig(al, off) + be.back();
    }
    // Hard locking: the leading nl columns, converged to the phase's lock
    // tolerance, are no longer filtered; the filtered rest is projected
    // against them and Rayleigh-Ritz runs on the rest only (nl as in LOBPCG
    // below).
    for (it = 0; it < o.maxit; ++it) {
      if ((s = residuals(nrm))) return s;
      for (int j = 0; j < n; ++j)
        if (!std::isfinite(nrm[j]))
          return fail(HELIC_ERR_NOCONV, "residual of column " + std::to_string(j) + " is not finite at iteration " +
                                            std::to_string(it));
      // the nev lowest by value (the locked prefix and the rest may interleave)
      double worst = 0.0;
      {
        const std::vector<int> ord = lowest_order();
        for (int q = 0; q < nev; ++q) worst = std::max(worst, nrm[ord[q]]);
      }
      if (worst <= o.tol && prec == HELIC_FP64) {
        converged = true;
        break;
      }
      const bool stagnant = stalled(worst);
      const bool to64 = prec != HELIC_FP64 && (worst <= switch_tol || (stagnant && prec == HELIC_FP32));
      const bool to32 = !to64 && prec == HELIC_BF16 && (worst <= switch_bf16 || stagnant);
      if ((to64 || to32) && o.stop_low) {
        stopped_low = true;
        break;
      }
      if (to64 || to32) {
        phase_best = HUGE_VAL;
        phase_stall = 0;
        // precision ladder: H X in the next precision and a fresh
        // Rayleigh-Ritz over every column (the locks of the lower phase are
        // released), then filters in that precision
        prec = to64 ? HELIC_FP64 : HELIC_FP32;
        nl = 0;
        if ((s = apply(S, AS, n))) return s;
        if ((s = rayleigh_ritz(0, n, n, 0))) return s;
        HIP_TRY_S(hipMemcpyAsync(S, Xn, sizeof(double) * Lc * n, hipMemcpyDeviceToDevice, st));
        HIP_TRY_S(hipMemcpyAsync(AS, AXn, sizeof(double) * Lc * n, hipMemcpyDeviceToDevice, st));
        --it;
        continue;
      }
      if (o.log_every > 0 && it % o.log_every == 0) {
        std::fprintf(stderr, "[helic] filter step %d: worst wanted residual %.3e, %d locked, %s H*X, %.1f s\n", it,
                     worst, nl, prec_name(), total.ms() / 1e3);
        std::fflush(stderr);
      }
      if (prec != HELIC_FP64) ++S_.iters_low;
      if (prec == HELIC_BF16) ++S_.iters_bf16;
      // in a low-precision phase a column is locked at its switch tolerance,
      // where filtering in that precision stops improving it; the next phase
      // starts unlocked
      const double lock_tol = phase_tol();
      while (nl < n - 1 && nrm[nl] <= lock_tol) ++nl;
      const int nu = n - nl;
      const int64_t nd = (int64_t)Lc * nu;
      const int gridc = (int)std::min<int64_t>(4096, (nd + NTS - 1) / NTS);
      double a = -HUGE_VAL, a0 = HUGE_VAL;
      for (int j = 0; j < n; ++j) {
        a = std::max(a, lam_h[j]);
        a0 = std::min(a0, lam_h[j]);
      }
      if (!(b_up > a)) return fail(HELIC_ERR_NOCONV, "spectrum bound does not exceed the Ritz values");
      const double e = 0.5 * (b_up - a), c = 0.5 * (b_up + a);
      double sigma = e / (a0 - c);
      const double tau = 2.0 / sigma;
      // Y1 = (H X - c X) sigma / e from the Rayleigh-Ritz block and its H X;
      // Y_i = (H Y_{i-1} - c Y_{i-1}) 2 sigma2 / e - sigma sigma2 Y_{i-2},
      // written over Y_{i-2}.  The coefficients of the m steps go to the
      // device first; the recurrence itself (m - 1 applications of H and m
      // elementwise steps) is the same launch sequence at every outer step
      // with the same locked count and precision, so it is captured once
      // into a HIP graph and replayed.
      double* const X0 = col(S, nl);
      double* const AX0 = col(AS, nl);
      for (int i = 1; i <= m; ++i) {
        if (i == 1) {
          cheb_h[0] = sigma / e;
          cheb_h[1] = c;
          cheb_h[2] = 0.0;
        } else {
          const double sigma2 = 1.0 / (tau - sigma);
          cheb_h[3 * (i - 1)] = 2.0 * sigma2 / e;
          cheb_h[3 * (i - 1) + 1] = c;
          cheb_h[3 * (i - 1) + 2] = -sigma * sigma2;
          sigma = sigma2;
        }
      }
      Timer tf;
      HIP_TRY_S(hipMemcpyAsync(cheb_d, cheb_h.data(), sizeof(double) * 3 * m, hipMemcpyHostToDevice, st));
      auto enqueue = [&]() -> helic_status {
        double* prev = X0;
        double* cur = col(S, n);
        hipLaunchKernelGGL(k_cheb_step_c, dim3(gridc), dim3(NTS), 0, st, AX0, X0, (const double*)nullptr, cur, nd,
                           (const double*)cheb_d);
        HIP_TRY_S(hipGetLastError());
        for (int i = 2; i <= m; ++i) {
          helic_status r = apply_H_impl(h, cur, L, AX0, L, nu, prec, st, chunk);
          if (r != HELIC_OK) return r;
          hipLaunchKernelGGL(k_cheb_step_c, dim3(gridc), dim3(NTS), 0, st, AX0, cur, prev, prev, nd,
                             (const double*)(cheb_d + 3 * (i - 1)));
          HIP_TRY_S(hipGetLastError());
          std::swap(prev, cur);
        }
        return HELIC_OK;
      };
      if (use_graph) {
        if (!fgraph.x || fgraph.nl != nl || fgraph.prec != prec) {
          fgraph.reset();
          // the intermediate buffer must not grow inside the capture
          if ((s = ensure_workspace(h, std::min(nu, chunk), slab_elem_bytes(prec) / 2))) return s;
          HIP_TRY_S(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          const helic_status r = enqueue();
          hipGraph_t g = nullptr;
          const hipError_t e2 = hipStreamEndCapture(st, &g);
          if (r != HELIC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
          }
          if (e2 != hipSuccess) return fail(HELIC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
          fgraph.g = g;
          HIP_TRY_S(hipGraphInstantiate(&fgraph.x, g, nullptr, nullptr, 0));
          fgraph.nl = nl;
          fgraph.prec = prec;
          ++S_.n_graphs;
        }
        HIP_TRY_S(hipGraphLaunch(fgraph.x, st));
      } else if ((s = enqueue())) {
        return s;
      }
      S_.n_apply += (int64_t)(m - 1) * nu;
      // the output block after m - 1 exchanges of the two work blocks
      double* cur = (m - 1) % 2 ? X0 : col(S, n);
      if ((s = sync())) return s;
      S_.t_apply_ms += tf.ms();
      Timer t;
      if (cur != X0) HIP_TRY_S(hipMemcpyAsync(X0, cur, sizeof(double) * nd, hipMemcpyDeviceToDevice, st));
      for (int rep = 0; rep < 2 && nl > 0; ++rep)
        if ((s = project(S, nullptr, nl, X0, nullptr, nu))) return s;
      int kept = 0;
      if ((s = ortho_block(X0, nullptr, nu, &kept))) return s;
      if (kept < nu) {
        // the filter collapsed directions: refill with random columns
        // orthogonal to the kept ones and the locked ones
        const int nk = nl + kept;
        const int64_t nr_ = (int64_t)Lc * (n - nk);
        hipLaunchKernelGGL(k_random_normal, dim3((int)std::min<int64_t>(4096, (nr_ + NTS - 1) / NTS)), dim3(NTS), 0,
                           st, col(S, nk), nr_, o.seed + 0x9e37ull * (uint64_t)(it + 1));
        HIP_TRY_S(hipGetLastError());
        for (int rep = 0; rep < 2; ++rep)
          if ((s = project(S, nullptr, nk, col(S, nk), nullptr, n - nk))) return s;
        int k2 = 0;
        if ((s = ortho_block(col(S, nk), nullptr, n - nk, &k2))) return s;
        if (k2 < n - nk) return fail(HELIC_ERR_NOCONV, "filtered block is rank deficient");
      }
      if ((s = sync())) return s;
      S_.t_rr_ms += t.ms();
      if ((s = apply(X0, AX0, nu))) return s;
      if ((s = rayleigh_ritz(nl, nu, nu, 0))) return s;
      HIP_TRY_S(hipMemcpyAsync(X0, col(Xn, nl), sizeof(double) * nd, hipMemcpyDeviceToDevice, st));
      HIP_TRY_S(hipMemcpyAsync(AX0, col(AXn, nl), sizeof(double) * nd, hipMemcpyDeviceToDevice, st));
    }
  } else {
    for (it = 0; it < o.maxit; ++it) {
      if ((s = residuals(nrm))) return s;
      for (int j = 0; j < n; ++j)
        if (!std::isfinite(nrm[j]))
          return fail(HELIC_ERR_NOCONV, "residual of column " + std::to_string(j) + " is not finite at iteration " +
                                            std::to_string(it));
      // the nev lowest by value (the locked prefix and the rest may interleave)
      bool all = true;
      double worst = 0.0;
      {
        const std::vector<int> ord = lowest_order();
        for (int q = 0; q < nev; ++q) {
          all = all && nrm[ord[q]] <= o.tol;
          worst = std::max(worst, nrm[ord[q]]);
        }
      }
      if (all && prec == HELIC_FP64) {
        converged = true;
        break;
      }
      const bool stagnant = stalled(worst);
      const bool to64 = prec != HELIC_FP64 && (worst <= switch_tol || (stagnant && prec == HELIC_FP32));
      const bool to32 = !to64 && prec == HELIC_BF16 && (worst <= switch_bf16 || stagnant);
      if ((to64 || to32) && o.stop_low) {
        stopped_low = true;
        break;
      }
      if (to64 || to32) {
        phase_best = HUGE_VAL;
        phase_stall = 0;
        // precision ladder: recompute H X and H P in the next precision and go on
        prec = to64 ? HELIC_FP64 : HELIC_FP32;
        exact_x = false;   // H X recomputed: X^H H X is no longer exactly diagonal
        if ((s = apply(S, AS, n))) return s;
        if ((s = apply(Pb, APb, np))) return s;
        --it;
        continue;
      }
      if (o.log_every > 0 && it % o.log_every == 0) {
        std::fprintf(stderr, "[helic] iteration %d: worst wanted residual %.3e, %s H*X, %.1f s\n", it, worst,
                     prec_name(), total.ms() / 1e3);
        std::fflush(stderr);
      }
      if (learned) {
        if (worst < best_worst) {
          best_worst = worst;
          stall = 0;
        } else if (++stall >= 3) {
          learned = false;
        }
      }
      if (prec != HELIC_FP64) ++S_.iters_low;
      if (prec == HELIC_BF16) ++S_.iters_bf16;
      // In a low-precision phase columns are locked at its switch tolerance:
      // iterating a column whose residual is at that precision's noise floor
      // makes its normalised update directions amplify the rounding
      // inconsistency between S and H S.
      const double lock_tol = phase_tol();
      if (prec == HELIC_FP64)
        while (nl < n - 1 && nrm[nl] <= o.tol) ++nl;
      active.clear();
      for (int j = nl; j < n; ++j)
        if (nrm[j] > lock_tol) active.push_back(j);
      const int na = (int)active.size();
      if (na == 0) return fail(HELIC_ERR_NOCONV, "no active column left below the target");
      // W = T(R_active) into S columns [n, n + na)
      Timer tp;
      HIP_TRY_S(hipMemcpyAsync(d_idx, active.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, st));
      double* W = col(S, n);
      hipLaunchKernelGGL(k_gather_cols, dim3(64, na), dim3(NTS), 0, st, R, W, d_idx, L, na);
      HIP_TRY_S(hipGetLastError());
      if (hv && it >= hv->next_iter && hv->ncol < hv->max_cols && (int)hv->snaps.size() < hv->n_snap) {
        if ((s = snapshot(it, active, W, na))) return s;
      }
      if (o.precond == 0 || (o.precond == 2 && !learned)) {
        if ((s = precondition_impl(h, W, L, W, L, na, st))) return s;
        if (o.precond == 2) ++S_.n_fallback;
      } else if (o.precond == 2) {
        std::vector<double> lam_a(na);
        for (int c = 0; c < na; ++c) lam_a[c] = lam_h[active[c]];
        HIP_TRY_S(hipMemcpyAsync(d, lam_a.data(), sizeof(double) * na, hipMemcpyHostToDevice, st));
        if ((s = lpc_precondition(h, W, L, d, W, L, na, st))) return s;
        if ((s = sync())) return s;   // lam_a is read by the copy above
      }
      if ((s = sync())) return s;
      S_.t_precond_ms += tp.ms();
      // W: project against X twice, orthonormalise, then apply H
      int nw = 0;
      {
        Timer t;
        for (int rep = 0; rep < 2; ++rep)
          if ((s = project(S, nullptr, n, W, nullptr, na))) return s;
        if ((s = ortho_block(W, nullptr, na, &nw))) return s;
        if ((s = sync())) return s;
        S_.t_rr_ms += t.ms();
      }
      if ((s = apply(W, col(AS, n), nw))) return s;
      // P after W: project against X and W twice, orthonormalise with H P
      int npk = 0;
      if (np > 0) {
        Timer t;
        double* P = col(S, n + nw);
        double* AP = col(AS, n + nw);
        HIP_TRY_S(hipMemcpyAsync(P, Pb, sizeof(double) * Lc * np, hipMemcpyDeviceToDevice, st));
        HIP_TRY_S(hipMemcpyAsync(AP, APb, sizeof(double) * Lc * np, hipMemcpyDeviceToDevice, st));
        // [X W] is orthonormal (W was projected against X and orthonormalised):
        // one projection against the joint block, twice
        for (int rep = 0; rep < 2; ++rep)
          if ((s = project(S, AS, n + nw, P, AP, np))) return s;
        if ((s = ortho_block(P, AP, np, &npk))) return s;
        if ((s = sync())) return s;
        S_.t_rr_ms += t.ms();
      }
      const int nx = n - nl;            // unlocked Ritz vectors
      const int k = nx + nw + npk;
      if ((s = rayleigh_ritz(nl, k, nx, exact_x ? nx : 0))) return s;
      exact_x = true;
      {
        Timer t;
        // new P = [W P] C[nx:k, active - nl], H P likewise
        rel.resize(na);
        for (int c = 0; c < na; ++c) rel[c] = active[c] - nl;
        HIP_TRY_S(hipMemcpyAsync(d_idx, rel.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_gather_sub, dim3((k - nx + 63) / 64, na), dim3(64), 0, st, C, kmax, nx, k - nx, d_idx,
                           na, T1, kmax);
        HIP_TRY_S(hipGetLastError());
        RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, na, k - nx, &one,
                             (const zc*)col(S, n), (int)L, (const zc*)T1, kmax, &zero, (zc*)Pb, (int)L));
        RB_TRY(rocblas_zgemm(rb, rocblas_operation_none, rocblas_operation_none, (int)L, na, k - nx, &one,
                             (const zc*)col(AS, n), (int)L, (const zc*)T1, kmax, &zero, (zc*)APb, (int)L));
        np = na;
        HIP_TRY_S(hipMemcpyAsync(col(S, nl), col(Xn, nl), sizeof(double) * Lc * nx, hipMemcpyDeviceToDevice, st));
        HIP_TRY_S(hipMemcpyAsync(col(AS, nl), col(AXn, nl), sizeof(double) * Lc * nx, hipMemcpyDeviceToDevice, st));
        if ((s = sync())) return s;   // rel is read by the copy above
        S_.t_rr_ms += t.ms();
      }
    }
  }
  if (!converged && (s = residuals(nrm))) return s;
  {
    // columns in ascending order of their Ritz values (locking may have
    // left them out of order)
    const std::vector<int> ord = lowest_order();
    std::vector<int32_t> ord32(ord.begin(), ord.end());
    HIP_TRY_S(hipMemcpyAsync(d_idx, ord32.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gather_cols, dim3(64, n), dim3(NTS), 0, st, S, Xn, d_idx, L, n);
    HIP_TRY_S(hipGetLastError());
    HIP_TRY_S(hipMemcpyAsync(S, Xn, sizeof(double) * Lc * n, hipMemcpyDeviceToDevice, st));
    if ((s = sync())) return s;
    std::vector<double> l2(n), r2(n);
    for (int q = 0; q < n; ++q) {
      l2[q] = lam_h[ord[q]];
      r2[q] = nrm[ord[q]];
    }
    lam_h.swap(l2);
    nrm.swap(r2);
  }
  if (!converged && !stopped_low) {
    converged = prec == HELIC_FP64;
    for (int j = 0; j < nev; ++j) converged = converged && nrm[j] <= o.tol;
  }
  if (stopped_low) converged = true;
  if (hv && converged && !stopped_low)
    if ((s = harvest_targets())) return s;
  if (evecs)
    HIP_TRY_S(hipMemcpy2DAsync(evecs, sizeof(double) * 2 * ldv, S, sizeof(double) * Lc, sizeof(double) * Lc, nev,
                               hipMemcpyDeviceToDevice, st));
  if ((s = sync())) return s;
  for (int j = 0; j < nev; ++j) {
    evals[j] = lam_h[j];
    resid[j] = nrm[j];
  }
  S_.iters = it;
  S_.t_total_ms = total.ms();
  if (stats) *stats = S_;
  if (!converged) return fail(HELIC_ERR_NOCONV, "iteration limit reached above tolerance");
  return HELIC_OK;
}

}  // namespace helic

using namespace helic;

extern "C" {

helic_status helic_eigensolve_ex(helic_basis h, const helic_solve_opts* o, double* evals, double* resid,
                                 double* evecs, int64_t ldv, helic_solve_stats* stats, void* stream) {
  if (!h || !o || !evals || !resid) return fail(HELIC_ERR_INVALID, "null argument");
  if (o->nev < 1 || o->nev > h->L || o->block < 1 || !(o->tol > 0) || o->maxit < 0 ||
      (evecs && ldv < h->L))
    return fail(HELIC_ERR_INVALID, "bad solver options");
  if (o->prec != HELIC_FP64 && o->prec != HELIC_FP32 && o->prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  if (o->precond < 0 || o->precond > 2) return fail(HELIC_ERR_UNSUPPORTED, "unknown preconditioner");
  if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "no potential set");
  if (o->precond == 2 && !lpc_attached(h)) return fail(HELIC_ERR_STATE, "no learned preconditioner attached");
  try {
    return eigensolve_impl(h, *o, evals, resid, evecs, ldv, stats, reinterpret_cast<hipStream_t>(stream), nullptr, 0,
                           true);
  } catch (const std::bad_alloc&) {
    return fail(HELIC_ERR_NOMEM, "host allocation failed");
  }
}

helic_status helic_eigensolve_chefsi(helic_basis h, const helic_solve_opts* o, int32_t degree, double* evals,
                                     double* resid, double* evecs, int64_t ldv, helic_solve_stats* stats,
                                     void* stream) {
  if (!h || !o || !evals || !resid) return fail(HELIC_ERR_INVALID, "null argument");
  if (o->nev < 1 || o->nev > h->L || o->block < 1 || !(o->tol > 0) || o->maxit < 0 ||
      (evecs && ldv < h->L) || degree < 0 || degree > 200)
    return fail(HELIC_ERR_INVALID, "bad solver options");
  if (o->prec != HELIC_FP64 && o->prec != HELIC_FP32 && o->prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "no potential set");
  try {
    return eigensolve_impl(h, *o, evals, resid, evecs, ldv, stats, reinterpret_cast<hipStream_t>(stream), nullptr,
                           degree > 0 ? degree : CHEB_DEGREE_AUTO, true);
  } catch (const std::bad_alloc&) {
    return fail(HELIC_ERR_NOMEM, "host allocation failed");
  }
}

helic_status helic_lpc_harvest(helic_basis h, const helic_solve_opts* o, int32_t n_snap, int32_t max_cols,
                               double* R, double* T, double* lam, int32_t* ncol, helic_solve_stats* stats,
                               void* stream) {
  if (!h || !o || !R || !T || !lam || !ncol) return fail(HELIC_ERR_INVALID, "null argument");
  *ncol = 0;
  if (n_snap < 1 || max_cols < 1) return fail(HELIC_ERR_INVALID, "bad harvest sizes");
  if (o->nev < 1 || o->nev > h->L || o->block < 1 || !(o->tol > 0) || o->maxit < 0)
    return fail(HELIC_ERR_INVALID, "bad solver options");
  if (o->prec != HELIC_FP64 && o->prec != HELIC_FP32 && o->prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  if (o->precond < 0 || o->precond > 2) return fail(HELIC_ERR_UNSUPPORTED, "unknown preconditioner");
  if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "no potential set");
  if (o->precond == 2 && !lpc_attached(h)) return fail(HELIC_ERR_STATE, "no learned preconditioner attached");
  try {
    Harvest hv;
    hv.n_snap = n_snap;
    hv.max_cols = max_cols;
    hv.R = R;
    hv.T = T;
    hv.lam = lam;
    std::vector<double> ev(o->nev), rs(o->nev);
    helic_status s = eigensolve_impl(h, *o, ev.data(), rs.data(), nullptr, 0, stats,
                                     reinterpret_cast<hipStream_t>(stream), &hv, 0, true);
    if (s) return s;
    *ncol = hv.ncol;
    return HELIC_OK;
  } catch (const std::bad_alloc&) {
    return fail(HELIC_ERR_NOMEM, "host allocation failed");
  }
}

helic_status helic_eigensolve(helic_basis h, int32_t nev, int32_t block, double tol, int32_t maxit, helic_prec prec,
                              uint64_t seed, double* evals, double* resid, double* evecs, int64_t ldv, int32_t* iters,
                              void* stream) {
  helic_solve_opts o;
  std::memset(&o, 0, sizeof(o));
  o.nev = nev;
  o.block = block;
  o.tol = tol;
  o.maxit = maxit;
  o.prec = prec;
  o.seed = seed;
  o.precond = 0;
  o.guard = -1;
  o.switch_tol = 1e-5;
  o.log_every = 0;
  helic_solve_stats st;
  std::memset(&st, 0, sizeof(st));
  helic_status s = helic_eigensolve_ex(h, &o, evals, resid, evecs, ldv, &st, stream);
  if (iters) *iters = st.iters;
  return s;
}

}  // extern "C"
