// Device-resident state of a basis handle.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace helic {

// Vectors per launch of the H*X stages; bounds the intermediate buffer to
// APPLY_CHUNK * n_r * n_modes complex values.
constexpr int APPLY_CHUNK = 64;
// States per real-space workspace pass of the density (n_t1*n_t2*n_r complex
// values each).
constexpr int DENSITY_CHUNK = 16;
// Chebyshev filter degree of the filtered eigensolver when the caller passes 0.
constexpr int CHEB_DEGREE_AUTO = 32;

struct SolverState;
}  // namespace helic
struct helic_lpc_s;
namespace helic {

struct DeviceState {
  int device = 0;
  DGroup* groups = nullptr;
  DMode* modes = nullptr;
  int32_t* row_ck = nullptr;
  double* kappa = nullptr;
  int32_t* rows1 = nullptr;
  double *tinv64 = nullptr, *tfwd64 = nullptr;
  float *tinv32 = nullptr, *tfwd32 = nullptr;
  uint16_t *tinv16 = nullptr, *tfwd16 = nullptr;   // BF16 tables (16x16x16 fragments)
  cplx<double>*tw1 = nullptr, *tw2 = nullptr;
  cplx<float>*tw1f = nullptr, *tw2f = nullptr;
  FftPlan plan1{}, plan2{};
  double* Vs = nullptr;
  float* Vsf = nullptr;
  bool have_potential = false;
  void* gh = nullptr;
  size_t gh_bytes = 0;
  // specialised angular stage (theta1 convolution with the spectrum of V)
  int fast_mpad = 0;              // 0: use the general angular kernel
  int fast_ntf = 256;
  int split_ntf = 0;              // > 0: the split theta1 FFT kernel serves this grid in FP32
                                  // arithmetic (its block size)
  bool pipe64 = false;            // FP64 angular stage by the two-vector pipeline k_angular_pipe
  int m_min = 0, m_count = 0;
  bool grid_var = false;          // the register-FFT angular kernel serves this grid
  int vchunk = 0;                 // (problem, radius, vector) items per workgroup of the specialised
                                  // angular kernels; 0: spread evenly over the resident workgroups
  int ang_slots64 = 1, ang_slots32 = 1, ang_slots16 = 1;   // resident workgroups of that kernel on the device
  int apply_chunk = APPLY_CHUNK;  // vectors per launch of the three stages
  int32_t* mode_pos = nullptr;    // mode -> (m - m_min) * ang_rs(n_t2) + ((n mod n_t2) ^ ang_swz)
  int32_t* blk_mode = nullptr;    // (m - m_min) * n_t2 + (n mod n_t2) -> mode, -1 if none
  double* Vh = nullptr;           // [n_r][n_t2][2 * fast_mpad - 1] complex
  float* Vhf = nullptr;
  DProb* probs64 = nullptr;       // one-entry problem tables of this handle
  DProb* probs32 = nullptr;
  DProb* probs16 = nullptr;       // BF16 mode: BF16 tables, FP32 potential
  double* part = nullptr;
  size_t part_bytes = 0;
  double* dens_ws = nullptr;      // density: real-space grids of one chunk of states
  size_t dens_ws_bytes = 0;
  double* dens_occ = nullptr;     // density: per-state weights
  size_t dens_occ_n = 0;
  // field derivatives: d xi / dr tables, a problem entry that uses them,
  // per-row factors 2 pi m and 2 pi n, radii, scaled-coefficient workspace
  double* tdinv64 = nullptr;
  DProb* probs_dr = nullptr;
  double* grad_fac = nullptr;
  double* rgrid = nullptr;
  double* grad_ws = nullptr;
  size_t grad_ws_bytes = 0;
  SolverState* solver = nullptr;
  // learned preconditioner: attached network, potential diagonal V_ii per
  // row (L values, then the n_r angular means; set with the potential),
  // per-call column workspace
  helic_lpc_s* lpc = nullptr;
  double* vdiag = nullptr;
  double* lpc_ws = nullptr;
  size_t lpc_ws_bytes = 0;
};

void release_solver_state(DeviceState* d);

// Everything one launch of the three H*X stages needs, for a single handle
// or a batch of grid-compatible handles.
struct LaunchSet {
  const DGroup* groups = nullptr;   // all groups of all problems (prob field set)
  int ngroups = 0;
  const DProb* probs64 = nullptr;
  const DProb* probs32 = nullptr;
  const DProb* probs16 = nullptr;
  int nprob = 1;
  int n_r = 0, n_t1 = 0, n_t2 = 0;
  size_t lds_inv64 = 0, lds_fwd64 = 0, lds_ang64 = 0, lds_fast64 = 0;   // FP32 uses half
  int fast_mpad = 0, fast_ntf = 256, split_ntf = 0, vchunk = 0;
  bool pipe64 = false;
  int rad_order = -1;                    // radial stages' work order (radial_item); -1: by precision
  int ang_slots64 = 1, ang_slots32 = 1, ang_slots16 = 1;
  bool grid_var = false;
  size_t lds_inv16 = 0, lds_fwd16 = 0;   // LDS bytes of the BF16 radial kernels
  int max_colpad = 0;                    // widest group's real columns, padded to 16
  int fwd_tm16 = 8;                      // register tiles per wave of the BF16 forward kernel
  int inv_ks = 24;                  // register k steps of the radial inverse stage
  int fwd_tmax = 4;                 // radial forward variant: register tiles per wave; 0, -1 = pipelined
                                    // with 2 or 4 staged columns per lane
  int fwd_tmax_plain = 4;           // the non-pipelined variant and its LDS bytes (FP64)
  size_t lds_fwd_plain64 = 0;
  size_t lds_fwd32 = 0;             // LDS bytes of the chosen forward variant in FP32
  bool kx_lds64 = false, kx_lds32 = false;   // pipelined forward stages kappa x in LDS
  int fwd_tm64 = 8, fwd_tm32 = 4;            // its register tiles per wave
  const int32_t* rows1 = nullptr;
  int nrows1 = 0;
  FftPlan plan1{}, plan2{};
  const void* tw1_64 = nullptr; const void* tw2_64 = nullptr;
  const void* tw1_32 = nullptr; const void* tw2_32 = nullptr;
  void* gh = nullptr;               // intermediate buffer (large enough for the call)
};

}  // namespace helic
