// Context internals shared by the C ABI sources (host code).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fft.h"
#include "particles.h"
#include "scan.h"

struct sbx_batch;

namespace sbx {

constexpr int kDiagCap = 4096;  // diagnostics records kept per context

struct Green {
  sbx_level geo;
  void* H;
  double rel_imag;
};

// One set of particle arrays (device, context precision).
struct PSet {
  void* x[3] = {};
  void* v[3] = {};
  void* m = nullptr;
  int8_t* comp = nullptr;
  int8_t* gal = nullptr;
  uint8_t* lost = nullptr;
  int32_t* id = nullptr;
};

LevelDev make_level(const sbx_level& s);
double q_crit_of(int n, double Rc, double Ro, double Rs);
bool same_level(const sbx_level& a, const sbx_level& b);
sbx_status validate(int ng, const sbx_hierarchy* h);
sbx_status dev_alloc(void** p, size_t bytes);
void free_ptr(void*& p);
sbx_status set_device(int dev);
void to_diag(const double* r, sbx_diag* d);

}  // namespace sbx

struct sbx_ctx {
  sbx_config cfg;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t esz = 4;  // bytes per real
  // particles: two sets, cur is the live one (device copy in d_cur)
  int64_t n = 0;
  sbx::PSet set[2];
  int cur = 0;
  bool bound = false;  // set[0] is the caller's storage (sbx_bind_device_particles)
  int* d_cur = nullptr;
  // grids
  bool built = false;
  int ngal = 0;
  int N = 0;
  sbx_hierarchy hh[sbx::kMaxGal];
  sbx::SysDev sys;
  int nslots[sbx::kMaxGal] = {};
  int slot_level[sbx::kMaxGal][sbx::kSlots] = {};
  void* grid_block = nullptr;  // all grids back to back
  size_t grid_elems = 0;
  size_t mass_elems = 0;       // the leading part of the block that takes masses
  bool fix_on = false;         // fixed-point mass assignment requested
  unsigned long long* fix = nullptr;  // its accumulators (mass_elems), while grids exist
  void* grid[sbx::kMaxGal][sbx::kSlots] = {};
  std::vector<sbx::Green> greens;
  void* X = nullptr;
  void* C = nullptr;
  int nsolves = 0;
  sbx::SolvePlan<float> plan32;
  sbx::SolvePlan<double> plan64;
  // adjoint grids (same layout as the grids) and their solve plan
  void* adj_block = nullptr;
  void* adj_work = nullptr;      // segment adjoint work arrays, kept between calls
  size_t adj_work_bytes = 0;
  sbx::SolvePlan<float> adj32;
  sbx::SolvePlan<double> adj64;
  // density-maximum centring: integer cell masses, search scratch, block sums
  unsigned long long* dm_hist = nullptr;
  size_t dm_elems = 0;
  unsigned long long* dm_aux = nullptr;
  double* dm_partial = nullptr;
  unsigned long long* dm_mmax = nullptr;  // largest particle mass (bits), taken at load
  // cell sort
  uint32_t* key = nullptr;
  uint32_t* rank = nullptr;
  uint32_t* count = nullptr;     // bins + 1
  uint32_t* scan_tmp = nullptr;
  size_t bins = 0;
  int sort_every = 4;
  int merge5 = 0;  // requested by sbx_set_outer_merge, applied at the next build
  // reductions and outputs
  double* centres = nullptr;       // kMaxGal * 3
  double* pre_partial = nullptr;   // (kRedBlocks + 1) * kPreVals
  double* com_partial = nullptr;   // kForceBlocksMax * kPreVals
  double* diag_partial = nullptr;  // kForceBlocksMax * kNDiag
  double* diag_one = nullptr;      // kNDiag
  double* diag_log = nullptr;      // kDiagCap * kNDiag
  int64_t diag_count = 0;
  double* acc = nullptr;           // n * 3, lazily
  double* pot = nullptr;           // n, lazily
  int64_t acc_n = 0;
  // state
  bool com_fresh = false;     // com_partial holds the current positions' sums
  bool solved = false;        // centres computed by a solve
  bool grids_fields = false;  // grids hold fields (not cell masses)
  int64_t step_count = 0;
  double dt_dev = 0.0;        // dt in the device instance record
  void* d_inst = nullptr;     // InstDev<T>, one record
  sbx_batch* batch = nullptr; // batch the context belongs to, if any
  sbx::Recorder rec;
};

// A group of contexts stepped together (one launch per phase, one HIP graph
// replay per step).
struct sbx_batch {
  std::vector<sbx_ctx*> ctx;
  int prec = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* d_inst = nullptr;          // InstDev<T>[n]
  int* d_cur = nullptr;            // live particle set per instance
  int cur = 0;                     // host mirror (all instances sort together)
  std::vector<sbx::InstInfo> info;
  uint32_t* counts = nullptr;      // all instances' sort counts, back to back
  size_t total_counts = 0;
  uint32_t* scan_tmp = nullptr;
  sbx::SolvePlan<float> p32;
  sbx::SolvePlan<double> p64;
  hipGraph_t graph[2] = {nullptr, nullptr};      // [0] plain step, [1] step with sort
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int sort_every = 4;
  int64_t step_count = 0;
  bool fresh = false;              // every instance's centre-of-mass sums are current
  bool pending = false;            // work queued since the last sbx_batch_sync
  std::vector<double> dt;
};

namespace sbx {

// Fill the instance record of a context (host copy) from its fields.
template <typename T>
InstDev<T> inst_of(const sbx_ctx* c);

// Upload the context's instance record (synchronises the context stream).
sbx_status upload_inst(sbx_ctx* c);

// Whether p is device memory of the given device.
bool on_device(const void* p, int device);
// Particle load (host or device arrays, host layout), read-back (caller's
// order) and borrowed-storage bind behind the ABI entry points.
sbx_status load_impl(sbx_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                     const int8_t* comp, const int8_t* gal, bool dev);
sbx_status get_impl(sbx_ctx* c, double* x, double* v, uint8_t* lost, bool dev);
sbx_status bind_impl(sbx_ctx* c, int64_t n, void* x, void* v, void* m, int8_t* comp, int8_t* gal,
                     uint8_t* lost);

inline InstInfo info_of(const sbx_ctx* c) {
  return InstInfo{c->n, c->mass_elems, c->dm_elems, c->fix != nullptr};
}

}  // namespace sbx
