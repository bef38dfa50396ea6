// Internal state of a basis handle, shared by the host set-up (basis.cpp) and
// the device code (device.hip, solver.hip).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/helic.h"

namespace helic {

// One angular mode (m, n) with its ragged radial length K (rows k = 1..K of
// the coefficient vector start at row0) and its DFT bin (m mod n_t1,
// n mod n_t2).
struct Mode {
  int32_t m, n, g;      // g = |n|
  int32_t K;            // number of k kept under the cutoff
  int64_t row0;         // first row of this mode in the compact order
  int32_t bin1, bin2;
};

// All modes whose radial functions have the same Bessel order share the
// radial tables xi_{g,k}(r_l) (at nu = 0: the modes of n = +-g / N).
struct Group {
  int32_t g;                // Bessel order |n N - nu|
  int32_t mode0, nmodes;    // modes [mode0, mode0 + nmodes) in compact order
  int32_t Kmax;
  int64_t row0, nrows;      // rows [row0, row0 + nrows) of the group
  int64_t tinv_off;         // offset (elements) of the packed inverse table
  int64_t tfwd_off;         // offset (elements) of the packed forward table
  int64_t tinv16_off;       // offsets (4-element fragments) of the BF16 tables
  int64_t tfwd16_off;
  std::vector<double> zeros;  // b_k^{g}, k = 1..Kmax
};

struct DeviceState;  // device.hip

}  // namespace helic

struct helic_basis_s {
  helic_params p;
  int64_t L = 0;
  int32_t n_t1 = 0, n_t2 = 0, n_r = 0;
  std::vector<helic::Mode> modes;
  std::vector<helic::Group> groups;
  std::vector<int32_t> mnk;       // L * 3
  std::vector<double> kappa;      // L
  std::vector<double> theta1, theta2, q, wq;
  std::vector<int32_t> row_ck;    // per row: (local mode index in group) << 16 | (k - 1)
  std::vector<int32_t> rows1;     // distinct theta1 bins that hold a mode
  // Packed radial tables (MFMA fragment order, see device.hip); doubles.
  std::vector<double> tab_inv, tab_fwd;
  std::vector<double> tab_dinv;   // d xi / dr in tab_inv's layout (App. C, field derivatives)
  // The same two tables in bfloat16 for the 16x16x16 BF16 MFMA: per group
  // fragments of 16 rows x 16 contraction indices, lane l holding row l % 16
  // and contraction indices 4 (l / 16) + 0..3 (four bfloat16 in 64 bits).
  std::vector<uint16_t> tab_inv16, tab_fwd16;
  int32_t max_kpad = 0, max_colpad = 0;   // LDS tile bounds over the groups
  std::vector<int32_t> fac1, fac2;        // radix factorisations of n_t1, n_t2
  helic::DeviceState* dev = nullptr;
};

namespace helic {
void set_error(const std::string& msg);
helic_status fail(helic_status s, const std::string& msg);
void device_release(helic_basis_s* h);   // device.hip
// Fragment packing used by both tables: tiles of 16 rows x 4 columns, 64
// entries per tile in MFMA lane order (lane l holds row 16 t + l % 16,
// column 4 s + l / 16).
constexpr int FRAG = 64;
}  // namespace helic
