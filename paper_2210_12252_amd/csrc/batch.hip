// Batches of problems (Bloch parameters of one or several structures, Sec.
// 3.3): per class of problems that share the grid and angular kernel variant,
// one launch per H*X stage over the ragged work of all its problems; all
// classes' launches captured in one HIP graph for replay; a tuner that picks,
// per class, the angular stage's work split, the radial inverse's register k
// steps and the radial forward variant (pipelined or plain, register tiles
// per wave) and records them; and concurrent eigensolves of all problems on a
// pool of streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "device_state.hpp"
#include "helic_internal.h"

namespace helic {

helic_status ensure_device(helic_basis_s* h);
DProb problem_entry(const helic_basis_s* h, bool fp64, int64_t Lpre, int64_t mpre);
DProb problem_entry16(const helic_basis_s* h, int64_t Lpre, int64_t mpre);
LaunchSet launch_set(const helic_basis_s* h);
template <typename T>
helic_status launch_stages(const LaunchSet& ls, const double* X, int64_t ldx, double* Y, int64_t ldy, int nvec,
                           hipStream_t st, int mode, hipEvent_t* ev);
struct Harvest;
helic_status eigensolve_impl(helic_basis_s* h, const helic_solve_opts& o, double* evals, double* resid,
                             double* evecs, int64_t ldv, helic_solve_stats* stats, hipStream_t st, Harvest* hv,
                             int cheb_degree, bool allow_graph);
void release_workspace(helic_basis_s* h);
size_t slab_elem_bytes(helic_prec prec);

}  // namespace helic

// Problems that share the grid and the angular kernel variant form a class;
// each class runs the three stages as one launch per stage over its problems'
// ragged work, the classes one after another on the same stream (they share
// the intermediate buffer).  Blocks stay concatenated over the whole batch.
struct BatchClass {
  std::vector<int> members;           // problem indices, ascending
  helic::DGroup* groups = nullptr;
  helic::DProb* probs64 = nullptr;
  helic::DProb* probs32 = nullptr;
  helic::DProb* probs16 = nullptr;
  int32_t* rows1 = nullptr;
  helic::LaunchSet ls;
  int64_t mtot = 0;                   // angular modes of the class's problems
  // tuner state: the variants it may choose between
  int inv_ks_min = 8;
  bool pf_ok = false;                 // every problem fits the pipelined forward kernel
  double tuned_ms = 0.0;
};

struct helic_batch_s {
  std::vector<helic_basis> bases;     // not owned
  int device = 0;
  std::vector<int64_t> Lpre;          // nprob + 1
  std::vector<BatchClass> classes;
  void* gh = nullptr;
  size_t gh_bytes = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int32_t> mirror;        // time reversal: partner solved in its place, or -1 (empty: none)
};

using namespace helic;

#define HIP_TRY_B(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(HELIC_ERR_HIP, std::string(#call) + " (batch): " + hipGetErrorString(e_)); \
  } while (0)

namespace {

template <typename T>
helic_status upload_vec(const std::vector<T>& v, T** d) {
  HIP_TRY_B(hipMalloc((void**)d, sizeof(T) * std::max<size_t>(v.size(), 1)));
  if (!v.empty()) HIP_TRY_B(hipMemcpy(*d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return HELIC_OK;
}

void release_graph(helic_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

helic_status batch_workspace(helic_batch_s* b, int nvec, size_t elem) {
  size_t need = 0;
  for (const BatchClass& c : b->classes) need = std::max(need, (size_t)nvec * c.ls.n_r * c.mtot * 2 * elem);
  if (need > b->gh_bytes) {
    release_graph(b);   // a captured graph refers to the old buffer
    if (b->gh) HIP_TRY_B(hipFree(b->gh));
    b->gh = nullptr;
    b->gh_bytes = 0;
    HIP_TRY_B(hipMalloc(&b->gh, need));
    b->gh_bytes = need;
  }
  for (BatchClass& c : b->classes) c.ls.gh = b->gh;
  return HELIC_OK;
}

helic_status class_launch(const BatchClass& c, const double* X, double* Y, int nvec, helic_prec prec,
                          hipStream_t st) {
  return prec == HELIC_FP64   ? launch_stages<double>(c.ls, X, -1, Y, -1, nvec, st, 1, nullptr)
         : prec == HELIC_FP32 ? launch_stages<float>(c.ls, X, -1, Y, -1, nvec, st, 1, nullptr)
                              : launch_stages<bf16x2>(c.ls, X, -1, Y, -1, nvec, st, 1, nullptr);
}

helic_status batch_launch(helic_batch_s* b, const double* X, double* Y, int nvec, helic_prec prec, hipStream_t st) {
  for (const BatchClass& c : b->classes) {
    const helic_status s = class_launch(c, X, Y, nvec, prec, st);
    if (s != HELIC_OK) return s;
  }
  return HELIC_OK;
}

helic_status check_block(helic_batch_s* b, const double* X, double* Y, int nvec, helic_prec prec) {
  if (!X || !Y || nvec < 1 || nvec > APPLY_CHUNK) return fail(HELIC_ERR_INVALID, "bad batch block (1 <= nvec <= 64)");
  if (prec != HELIC_FP64 && prec != HELIC_FP32 && prec != HELIC_BF16)
    return fail(HELIC_ERR_UNSUPPORTED, "unknown precision");
  const char* a = reinterpret_cast<const char*>(X);
  const char* c = reinterpret_cast<const char*>(Y);
  const size_t n = (size_t)nvec * b->Lpre.back() * 16;
  if (a < c + n && c < a + n) return fail(HELIC_ERR_INVALID, "X and Y overlap");
  return HELIC_OK;
}

void release_class(BatchClass& c) {
  void* ptrs[] = {c.groups, c.probs64, c.probs32, c.probs16, c.rows1};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  c.groups = nullptr;
  c.probs64 = c.probs32 = c.probs16 = nullptr;
  c.rows1 = nullptr;
}

// Device tables and launch parameters of one class (problem offsets Lpre
// over the whole batch, slab offsets within the class).
helic_status build_class(helic_batch_s* b, BatchClass& cl) {
  const helic_basis_s* h0 = b->bases[cl.members[0]];
  const int np = (int)cl.members.size();
  std::vector<DGroup> groups;
  std::vector<DProb> p64(np), p32(np), p16(np);
  std::vector<char> row_used(h0->n_t1, 0);
  int64_t mpre = 0;
  size_t lds_inv = 0, lds_fwd = 0, lds_ang = 0, lds_fwd_plain = 0, lds_fwd32 = 0, lds_inv16 = 0, lds_fwd16 = 0;
  bool kx64 = true, kx32 = true;
  int tm64 = 4, tm32 = 4, tm16 = 8;
  int fwd_tmax_plain = 4, inv_ks = 8, max_colpad = 0;
  bool all_pf = true, pf_wide = false;
  for (int i = 0; i < np; ++i) {
    const int p = cl.members[i];
    const helic_basis_s* h = b->bases[p];
    p64[i] = problem_entry(h, true, b->Lpre[p], mpre);
    p32[i] = problem_entry(h, false, b->Lpre[p], mpre);
    p16[i] = problem_entry16(h, b->Lpre[p], mpre);
    for (const Group& g : h->groups)
      groups.push_back(DGroup{g.mode0, g.nmodes, g.Kmax, i, g.row0, g.nrows, g.tinv_off, g.tfwd_off, g.tinv16_off,
                              g.tfwd16_off});
    for (int r : h->rows1) row_used[r] = 1;
    mpre += (int64_t)h->modes.size();
    const LaunchSet one = launch_set(h);
    lds_inv = std::max(lds_inv, one.lds_inv64);
    lds_inv16 = std::max(lds_inv16, one.lds_inv16);
    lds_fwd16 = std::max(lds_fwd16, one.lds_fwd16);
    max_colpad = std::max(max_colpad, one.max_colpad);
    tm16 = std::max(tm16, one.fwd_tm16);
    lds_fwd = std::max(lds_fwd, one.lds_fwd64);
    lds_fwd32 = std::max(lds_fwd32, one.lds_fwd32);
    kx64 = kx64 && one.kx_lds64;
    kx32 = kx32 && one.kx_lds32;
    tm64 = std::max(tm64, one.fwd_tm64);
    tm32 = std::max(tm32, one.fwd_tm32);
    lds_fwd_plain = std::max(lds_fwd_plain, one.lds_fwd_plain64);
    lds_ang = std::max(lds_ang, one.lds_ang64);
    fwd_tmax_plain = std::max(fwd_tmax_plain, one.fwd_tmax_plain);
    inv_ks = std::max(inv_ks, one.inv_ks);
    all_pf = all_pf && one.fwd_tmax <= 0;
    pf_wide = pf_wide || one.fwd_tmax < 0;
  }
  cl.mtot = mpre;
  std::vector<int32_t> rows1;
  for (int i = 0; i < h0->n_t1; ++i)
    if (row_used[i]) rows1.push_back(i);
  helic_status s;
  if ((s = upload_vec(groups, &cl.groups)) || (s = upload_vec(p64, &cl.probs64)) ||
      (s = upload_vec(p32, &cl.probs32)) || (s = upload_vec(p16, &cl.probs16)) || (s = upload_vec(rows1, &cl.rows1)))
    return s;
  LaunchSet& ls = cl.ls;
  ls = launch_set(h0);
  ls.groups = cl.groups;
  ls.ngroups = (int)groups.size();
  ls.probs64 = cl.probs64;
  ls.probs32 = cl.probs32;
  ls.probs16 = cl.probs16;
  ls.nprob = np;
  ls.lds_inv64 = lds_inv;
  ls.lds_inv16 = lds_inv16;
  ls.lds_fwd16 = lds_fwd16;
  ls.max_colpad = max_colpad;
  ls.fwd_tm16 = tm16;
  // the pipelined radial forward variant only if every problem fits it
  ls.inv_ks = inv_ks;
  ls.fwd_tmax = all_pf ? (pf_wide ? -1 : 0) : fwd_tmax_plain;
  ls.fwd_tmax_plain = fwd_tmax_plain;
  ls.lds_fwd_plain64 = lds_fwd_plain;
  ls.lds_fwd64 = all_pf ? lds_fwd : lds_fwd_plain;
  ls.lds_fwd32 = all_pf ? lds_fwd32 : lds_fwd_plain / 2;
  ls.kx_lds64 = all_pf && kx64;
  ls.kx_lds32 = all_pf && kx32;
  ls.fwd_tm64 = tm64;
  ls.fwd_tm32 = tm32;
  ls.lds_ang64 = lds_ang + rows1.size() * sizeof(int32_t);
  ls.rows1 = cl.rows1;
  ls.nrows1 = (int)rows1.size();
  ls.gh = nullptr;
  cl.inv_ks_min = inv_ks;
  cl.pf_ok = all_pf;
  return HELIC_OK;
}

// Mean time (ms) of one class's three stages over 5 launches after 2 warm ones.
helic_status time_class(const BatchClass& c, const double* X, double* Y, int nvec, helic_prec prec, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1, double* ms) {
  helic_status s = HELIC_OK;
  for (int rep = 0; rep < 2 && s == HELIC_OK; ++rep) s = class_launch(c, X, Y, nvec, prec, st);
  if (s != HELIC_OK) return s;
  HIP_TRY_B(hipEventRecord(e0, st));
  for (int rep = 0; rep < 5 && s == HELIC_OK; ++rep) s = class_launch(c, X, Y, nvec, prec, st);
  HIP_TRY_B(hipEventRecord(e1, st));
  HIP_TRY_B(hipEventSynchronize(e1));
  float t = 0;
  HIP_TRY_B(hipEventElapsedTime(&t, e0, e1));
  *ms = t / 5.0;
  return s;
}

// Forward-stage variants of a class: pipelined with 8 or 4 register tiles
// per wave (where every problem fits it), or the plain kernel with 4 or 8.
struct FwdVariant {
  int tmax, tm;
};

void set_forward(BatchClass& c, const FwdVariant& v, const size_t lds_pf64, const size_t lds_pf32, bool kx64,
                 bool kx32) {
  LaunchSet& ls = c.ls;
  if (v.tmax <= 0) {
    ls.fwd_tmax = v.tmax;
    ls.fwd_tm64 = ls.fwd_tm32 = v.tm;
    ls.lds_fwd64 = lds_pf64;
    ls.lds_fwd32 = lds_pf32;
    ls.kx_lds64 = kx64;
    ls.kx_lds32 = kx32;
  } else {
    ls.fwd_tmax = v.tm;
    ls.lds_fwd64 = ls.lds_fwd_plain64;
    ls.lds_fwd32 = ls.lds_fwd_plain64 / 2;
    ls.kx_lds64 = ls.kx_lds32 = false;
  }
}

// Tunes one class on the batch's buffers: the angular work split, the
// radial inverse's register k steps and the radial forward variant, one
// knob at a time, each against the whole class's three stages.
helic_status tune_class(BatchClass& c, const double* X, double* Y, int nvec, helic_prec prec, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
  double best = 0.0;
  helic_status s = time_class(c, X, Y, nvec, prec, st, e0, e1, &best);
  if (s != HELIC_OK) return s;
  auto trial = [&](auto apply, auto undo) -> helic_status {
    apply();
    double ms = 0.0;
    helic_status r = time_class(c, X, Y, nvec, prec, st, e0, e1, &ms);
    if (r != HELIC_OK) return r;
    if (ms < best) best = ms;
    else undo();
    return HELIC_OK;
  };
  if (c.ls.fast_mpad || c.ls.grid_var) {
    for (int v : {0, 2, 4, 8, 16}) {
      const int old = c.ls.vchunk;
      if (v == old) continue;
      if ((s = trial([&] { c.ls.vchunk = v; }, [&] { c.ls.vchunk = old; }))) return s;
    }
  }
  if (prec != HELIC_BF16) {
    for (int ks : {c.inv_ks_min, 24}) {
      const int old = c.ls.inv_ks;
      if (ks == old) continue;
      if ((s = trial([&] { c.ls.inv_ks = ks; }, [&] { c.ls.inv_ks = old; }))) return s;
    }
    const size_t pf64 = c.ls.lds_fwd64, pf32 = c.ls.lds_fwd32;
    const bool kx64 = c.ls.kx_lds64, kx32 = c.ls.kx_lds32;
    const int cb = c.ls.fwd_tmax;   // 0 or -1 when pipelined
    std::vector<FwdVariant> cands;
    if (c.pf_ok) cands = {{cb, 8}, {cb, 4}, {4, 4}, {4, 8}};
    else cands = {{4, 4}, {4, 8}};
    FwdVariant cur{c.ls.fwd_tmax, c.ls.fwd_tmax <= 0 ? (prec == HELIC_FP64 ? c.ls.fwd_tm64 : c.ls.fwd_tm32)
                                                     : c.ls.fwd_tmax};
    for (const FwdVariant& v : cands) {
      if (v.tmax == cur.tmax && v.tm == cur.tm) continue;
      const FwdVariant keep = cur;
      if ((s = trial([&] { set_forward(c, v, pf64, pf32, kx64, kx32); cur = v; },
                     [&] { set_forward(c, keep, pf64, pf32, kx64, kx32); cur = keep; })))
        return s;
    }
  }
  c.tuned_ms = best;
  return HELIC_OK;
}

}  // namespace

extern "C" {

helic_status helic_batch_create(const helic_basis* bases, int32_t nprob, helic_batch* out) {
  if (!bases || !out || nprob < 1) return fail(HELIC_ERR_INVALID, "bad arguments");
  *out = nullptr;
  const helic_basis_s* h0 = bases[0];
  if (!h0) return fail(HELIC_ERR_INVALID, "null handle");
  for (int p = 0; p < nprob; ++p) {
    const helic_basis_s* h = bases[p];
    if (!h) return fail(HELIC_ERR_INVALID, "null handle");
    if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "every problem needs a potential first");
    if (h->dev->device != h0->dev->device) return fail(HELIC_ERR_INVALID, "problems of a batch must share the device");
  }
  helic_batch_s* b = new helic_batch_s();
  b->bases.assign(bases, bases + nprob);
  b->device = h0->dev->device;
  b->Lpre.assign(nprob + 1, 0);
  for (int p = 0; p < nprob; ++p) {
    const helic_basis_s* h = bases[p];
    b->Lpre[p + 1] = b->Lpre[p] + h->L;
    // class: same grid and angular kernel variant
    int ci = -1;
    for (size_t c = 0; c < b->classes.size() && ci < 0; ++c) {
      const helic_basis_s* g = bases[b->classes[c].members[0]];
      if (g->n_t1 == h->n_t1 && g->n_t2 == h->n_t2 && g->n_r == h->n_r && g->dev->fast_mpad == h->dev->fast_mpad &&
          g->dev->fast_ntf == h->dev->fast_ntf && g->dev->split_ntf == h->dev->split_ntf &&
          g->dev->pipe64 == h->dev->pipe64 &&
          g->dev->grid_var == h->dev->grid_var)
        ci = (int)c;
    }
    if (ci < 0) {
      b->classes.emplace_back();
      ci = (int)b->classes.size() - 1;
    }
    b->classes[ci].members.push_back(p);
  }
  for (BatchClass& c : b->classes) {
    const helic_status s = build_class(b, c);
    if (s != HELIC_OK) {
      helic_batch_destroy(b);
      return s;
    }
  }
  *out = b;
  return HELIC_OK;
}

helic_status helic_batch_destroy(helic_batch b) {
  if (!b) return HELIC_OK;
  release_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (BatchClass& c : b->classes) release_class(c);
  if (b->gh) (void)hipFree(b->gh);
  delete b;
  return HELIC_OK;
}

helic_status helic_batch_info(helic_batch b, int64_t* offsets) {
  if (!b || !offsets) return fail(HELIC_ERR_INVALID, "null argument");
  std::copy(b->Lpre.begin(), b->Lpre.end(), offsets);
  return HELIC_OK;
}

helic_status helic_batch_classes(helic_batch b, int32_t* nclasses, int32_t* class_of) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  if (nclasses) *nclasses = (int32_t)b->classes.size();
  if (class_of)
    for (size_t c = 0; c < b->classes.size(); ++c)
      for (int p : b->classes[c].members) class_of[p] = (int32_t)c;
  return HELIC_OK;
}

helic_status helic_batch_apply(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec,
                               void* stream) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  helic_status s = check_block(b, X, Y, nvec, prec);
  if (s != HELIC_OK) return s;
  if ((s = batch_workspace(b, nvec, slab_elem_bytes(prec) / 2))) return s;
  return batch_launch(b, X, Y, nvec, prec, reinterpret_cast<hipStream_t>(stream));
}

helic_status helic_batch_capture(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  helic_status s = check_block(b, X, Y, nvec, prec);
  if (s != HELIC_OK) return s;
  if ((s = batch_workspace(b, nvec, slab_elem_bytes(prec) / 2))) return s;
  release_graph(b);
  if (!b->cap_stream) HIP_TRY_B(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIP_TRY_B(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  s = batch_launch(b, X, Y, nvec, prec, b->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (s != HELIC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(HELIC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  b->graph = g;
  HIP_TRY_B(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return HELIC_OK;
}

helic_status helic_batch_replay(helic_batch b, void* stream) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  if (!b->exec) return fail(HELIC_ERR_STATE, "no captured graph");
  HIP_TRY_B(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
  return HELIC_OK;
}

helic_status helic_batch_tune_classes(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec,
                                      void* stream, helic_batch_class_tuning* out, int32_t max_classes,
                                      int32_t* nclasses) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  helic_status s = check_block(b, X, Y, nvec, prec);
  if (s != HELIC_OK) return s;
  if ((s = batch_workspace(b, nvec, slab_elem_bytes(prec) / 2))) return s;
  release_graph(b);   // a captured graph holds the old launch parameters
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIP_TRY_B(hipEventCreate(&e0));
  HIP_TRY_B(hipEventCreate(&e1));
  for (BatchClass& c : b->classes)
    if ((s = tune_class(c, X, Y, nvec, prec, st, e0, e1)) != HELIC_OK) break;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != HELIC_OK) return s;
  if (nclasses) *nclasses = (int32_t)b->classes.size();
  for (int c = 0; out && c < (int)b->classes.size() && c < max_classes; ++c) {
    const BatchClass& cl = b->classes[c];
    helic_batch_class_tuning& t = out[c];
    t.n_t1 = cl.ls.n_t1;
    t.n_t2 = cl.ls.n_t2;
    t.n_r = cl.ls.n_r;
    t.nprob = (int32_t)cl.members.size();
    t.items_per_wg = cl.ls.vchunk;
    t.inv_ksteps = prec == HELIC_BF16 ? 4 * ((4 * cl.ls.inv_ks + 15) / 16) : cl.ls.inv_ks;
    t.fwd_pipelined = cl.ls.fwd_tmax <= 0 ? 1 : 0;
    t.fwd_tiles = prec == HELIC_BF16 ? cl.ls.fwd_tm16
                  : cl.ls.fwd_tmax <= 0 ? (prec == HELIC_FP64 ? cl.ls.fwd_tm64 : cl.ls.fwd_tm32)
                                        : cl.ls.fwd_tmax;
    t.ms = cl.tuned_ms;
  }
  return HELIC_OK;
}

helic_status helic_batch_tune(helic_batch b, const double* X, double* Y, int32_t nvec, helic_prec prec, void* stream,
                              int32_t* chosen, double* ms_best) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  helic_status s = helic_batch_tune_classes(b, X, Y, nvec, prec, stream, nullptr, 0, nullptr);
  if (s != HELIC_OK) return s;
  if (chosen) *chosen = b->classes[0].ls.vchunk;
  if (ms_best) {
    double t = 0.0;
    for (const BatchClass& c : b->classes) t += c.tuned_ms;
    *ms_best = t;
  }
  return HELIC_OK;
}

static helic_status batch_eigensolve(helic_batch b, const helic_solve_opts* o, int cheb_degree, int32_t nstreams,
                                     double* evals, double* resid, helic_solve_stats* stats, int32_t* status) {
  if (!b || !o || !evals || !resid || nstreams < 1) return fail(HELIC_ERR_INVALID, "bad arguments");
  const int nprob = (int)b->bases.size();
  for (helic_basis h : b->bases)
    if (o->nev < 1 || o->nev > h->L) return fail(HELIC_ERR_INVALID, "nev out of range for a problem");
  std::atomic<int> next(0);
  std::vector<helic_status> st(nprob, HELIC_OK);
  std::vector<std::string> msg(nprob);
  const bool tr = !b->mirror.empty();
  auto worker = [&]() {
    (void)hipSetDevice(b->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    for (;;) {
      const int p = next.fetch_add(1);
      if (p >= nprob) break;
      if (tr && b->mirror[p] >= 0) continue;   // takes its time-reversal partner's results below
      helic_solve_stats ss;
      std::memset(&ss, 0, sizeof(ss));
      st[p] = s ? eigensolve_impl(b->bases[p], *o, evals + (size_t)p * o->nev, resid + (size_t)p * o->nev, nullptr, 0,
                                  &ss, s, nullptr, cheb_degree, false)
                : HELIC_ERR_HIP;
      if (st[p] != HELIC_OK) msg[p] = helic_last_error();
      if (stats) stats[p] = ss;
      // keep device memory bounded by the number of concurrent solves
      if (s) (void)hipStreamSynchronize(s);
      release_workspace(b->bases[p]);
    }
    if (s) (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  const int nt = std::min(nstreams, nprob);
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  // time-reversal partners: lambda_j(eta, nu) = lambda_j(-eta, N - nu) (Sec. 3.3)
  for (int p = 0; tr && p < nprob; ++p) {
    const int q = b->mirror[p];
    if (q < 0) continue;
    std::copy(evals + (size_t)q * o->nev, evals + (size_t)(q + 1) * o->nev, evals + (size_t)p * o->nev);
    std::copy(resid + (size_t)q * o->nev, resid + (size_t)(q + 1) * o->nev, resid + (size_t)p * o->nev);
    st[p] = st[q];
    msg[p] = msg[q];
    if (stats) std::memset(&stats[p], 0, sizeof(helic_solve_stats));   // nothing was solved for p
  }
  helic_status ret = HELIC_OK;
  for (int p = 0; p < nprob; ++p) {
    if (status) status[p] = st[p];
    if (st[p] != HELIC_OK && st[p] != HELIC_ERR_NOCONV && ret == HELIC_OK) {
      ret = fail(st[p], "problem " + std::to_string(p) + ": " + msg[p]);
    }
  }
  if (ret == HELIC_OK)
    for (int p = 0; p < nprob; ++p)
      if (st[p] == HELIC_ERR_NOCONV) return fail(HELIC_ERR_NOCONV, "problem " + std::to_string(p) + " did not converge");
  return ret;
}

helic_status helic_batch_time_reversal(helic_batch b, int32_t enable, int32_t* npairs) {
  if (!b) return fail(HELIC_ERR_INVALID, "null batch");
  if (npairs) *npairs = 0;
  b->mirror.clear();
  if (!enable) return HELIC_OK;
  const int nprob = (int)b->bases.size();
  std::vector<int32_t> mirror(nprob, -1);
  std::vector<std::vector<double>> V(nprob);
  auto potential = [&](int p) -> helic_status {
    if (!V[p].empty()) return HELIC_OK;
    const helic_basis h = b->bases[p];
    if (!h->dev || !h->dev->have_potential) return fail(HELIC_ERR_STATE, "a problem of the batch has no potential");
    V[p].resize((size_t)h->n_t1 * h->n_t2 * h->n_r);
    HIP_TRY_B(hipMemcpy(V[p].data(), h->dev->Vs, sizeof(double) * V[p].size(), hipMemcpyDeviceToHost));
    return HELIC_OK;
  };
  int pairs = 0;
  for (int p = 0; p < nprob; ++p) {
    const helic_params& a = b->bases[p]->p;
    // partner (-eta, (N - nu) mod N), with eta = -1/2 its own negative
    const double eta_p = a.eta <= -0.5 ? a.eta : -a.eta;
    if (eta_p == a.eta && (2 * a.nu) % a.ncyc == 0) continue;   // its own partner
    for (int q = 0; q < p; ++q) {
      const helic_params& c = b->bases[q]->p;
      if (mirror[q] >= 0 || std::fabs(c.eta - eta_p) > 1e-12 || a.R != c.R || a.tau != c.tau ||
          a.alpha != c.alpha || a.ecut != c.ecut || a.ncyc != c.ncyc || c.nu != (a.ncyc - a.nu) % a.ncyc ||
          a.m_max != c.m_max ||
          a.n_max != c.n_max || a.k_max != c.k_max || b->bases[p]->L != b->bases[q]->L ||
          b->bases[p]->n_r != b->bases[q]->n_r)
        continue;
      bool taken = false;
      for (int p2 = 0; p2 < p; ++p2) taken = taken || mirror[p2] == q;
      if (taken) continue;
      helic_status s;
      if ((s = potential(p)) || (s = potential(q))) return s;
      if (V[p] != V[q]) continue;   // the same structure only
      mirror[p] = q;
      ++pairs;
      break;
    }
  }
  b->mirror = mirror;
  if (npairs) *npairs = pairs;
  return HELIC_OK;
}

helic_status helic_batch_eigensolve(helic_batch b, const helic_solve_opts* o, int32_t nstreams, double* evals,
                                    double* resid, helic_solve_stats* stats, int32_t* status) {
  return batch_eigensolve(b, o, 0, nstreams, evals, resid, stats, status);
}

helic_status helic_batch_eigensolve_chefsi(helic_batch b, const helic_solve_opts* o, int32_t degree,
                                           int32_t nstreams, double* evals, double* resid,
                                           helic_solve_stats* stats, int32_t* status) {
  if (degree < 0 || degree > 200) return fail(HELIC_ERR_INVALID, "bad filter degree");
  return batch_eigensolve(b, o, degree > 0 ? degree : CHEB_DEGREE_AUTO, nstreams, evals, resid, stats, status);
}

}  // extern "C"
