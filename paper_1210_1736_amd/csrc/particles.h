// Particle-side kernels of the nested-grid PM step (host interface).
//
// Every launch covers a set of independent instances (a context is one
// instance; a batch of contexts is several) described by a device array of
// InstDev records; instance i owns the blocks [span.start[i], span.start[i+1]).
#pragma once

#include <vector>

#include "common.h"

namespace sbx {

constexpr int kMaxGal = 8;       // galaxies per instance
constexpr int kSlots = 7;        // grids per 3-level galaxy (5 fields + 2 mass-only)
constexpr int kFieldSlots = 5;   // solved grids per 3-level galaxy
constexpr int kSlotG2 = 5;       // grid 2 masses (core, middle level)
constexpr int kSlotG4 = 6;       // grid 4 masses (core and ring, global level)
constexpr int kNComp = 8;        // particle component ids
constexpr int kMaxInst = 32;     // instances per launch
// diagnostics record: per component [ekin, epot, Lx, Ly, Lz, count],
// disc [sum vR, sum vR^2, sum vz, sum vz^2, count], lost count
constexpr int kDiagComp = 6;
constexpr int kDiagDisc = kNComp * kDiagComp;
constexpr int kDiagLost = kDiagDisc + 5;
constexpr int kNDiag = kDiagLost + 1;
constexpr int kPreVals = kMaxGal * 4;  // per galaxy [m, m x, m y, m z]
constexpr int kRedBlocks = 1024;       // blocks per instance of the loss-test / COM pass
constexpr int kForceBlocksMax = 2048;  // blocks per instance of the force pass
constexpr int kDepChunk = 8192;        // particles per block of the mass assignment
constexpr int kArgParts = 256;         // blocks per galaxy of the densest-cell search

// One grid geometry as the kernels use it (all float64, computed on the host
// exactly as the method's formulas read: l = 2R/(N-4), lz = q l, gamma = 1/l).
struct LevelDev {
  int N;
  double half;   // N/2
  double l, lz;  // cell lengths x/y and z
  double gx, gz; // 1/l, 1/lz
  double inv_q;  // 1/q
  double R2;     // R*R
  // Eq. 8 coefficients: 1/(2l), 1/(2lz), 1/l^2, 1/lz^2, 1/(4 l l), 1/(4 l lz)
  double c_2l, c_2lz, c_l2, c_lz2, c_4ll, c_4llz;
};

struct HierDev {
  int n_levels;
  int centring;  // 0 fixed, 1 centre of mass, 2 density maximum
  LevelDev lv[3];
  double centre[3];   // fixed centre (inner/middle levels, or the single grid)
  double outer_c[3];  // centre of the global grid (3 levels)
};

struct SysDev {
  int ngal;
  int taylor;
  int merge5;  // grid 5 of every galaxy summed into galaxy 0's slot 3 (one solve)
  HierDev h[kMaxGal];
};

template <typename T>
struct PartDev {
  T* x[3];
  T* v[3];
  T* m;
  int8_t* comp;
  int8_t* gal;
  uint8_t* lost;
  int32_t* id;   // caller's index of the particle held in this slot
  int64_t n;
};

// Grid slots of one galaxy: 3 levels -> 0: grid 1 (inner, core),
// 1: grid 3 (middle, ring), 2: grids 2+3 (middle, core+ring), 3: grid 5
// (global, outer), 4: grids 4+5 (global, all), 5: grid 2 masses, 6: grid 4
// masses.  Particles deposit into 0, 1, 3, 5 and 6 (each mass once); the
// solves of slots 2 and 4 read 5 + 1 and 6 + 3 and write their fields into
// slots 2 and 4.  1 level -> slot 0 only.  With merge5: slot 3 of galaxy 0
// holds grid 5 of all galaxies summed, slot 3 of the others is unused, and
// slot 4 is the field of grid 4 alone.
template <typename T>
struct GridsDev {
  T* g[kMaxGal][kSlots];
};

template <typename T>
struct InstDev {
  PartDev<T> p[2];          // two particle sets; cur[i] selects the live one
  SysDev sys;
  GridsDev<T> G;
  double* centres;          // 3 * kMaxGal
  double* com_partial;      // kPreVals columns of kForceBlocksMax block rows (column-major)
  double* pre_partial;      // kPreVals columns of kRedBlocks block rows (column-major)
  double* diag_partial;     // force_blocks(n) rows of kNDiag
  double* diag_out;         // kNDiag: where the next diagnostics record goes
  double* acc;              // n * 3 (write mode)
  double* pot;              // n (write mode, physical potential)
  T* grid_block;            // all grids of the instance, back to back
  size_t grid_elems;        // the leading grids that take masses (cleared per step)
  unsigned long long* fix;  // fixed-point mass accumulators, grid_elems of them (null: FP sums)
  uint32_t* key;            // n
  uint32_t* rank;           // n: place of the particle within its sort bin
  uint32_t* count;          // bins + 1: this instance's slice of the shared counts
  uint32_t part_base;       // sort position of the instance's first particle
  // density-maximum centring (null / 0 when no galaxy uses it)
  unsigned long long* dm_hist;  // ngal * N^3 integer cell masses of the inner grids
  size_t dm_elems;
  unsigned long long* dm_aux;   // [g] densest cell of galaxy g (all ones: none), then
                                // kMaxGal * kArgParts (value, index) partials
  double* dm_partial;           // as pre_partial: block sums around the densest cell
  const unsigned long long* dm_mmax;  // bits of the largest particle mass (set at load)
  double dt;
  int64_t n;
};
constexpr int kDmAux = kMaxGal + 2 * kMaxGal * kArgParts;

// Counting-sort bins.  A particle's bin is the cell of its finest grid
// relative to its own galaxy; bins are ordered by galaxy, level, z, y, x,
// and the last bin holds the lost particles.  (Coarser bins shorten the sort
// but change the order the deposit sees, which costs it more than the sort
// saves.)
__host__ __device__ inline size_t level_bins(const HierDev& h, int lev) {
  const size_t n = (size_t)h.lv[lev].N;
  return n * n * n;
}
__host__ __device__ inline size_t bins_before(const SysDev& s, int g, int lev) {
  size_t b = 0;
  for (int gg = 0; gg < g; ++gg)
    for (int l = 0; l < s.h[gg].n_levels; ++l) b += level_bins(s.h[gg], l);
  for (int l = 0; l < lev; ++l) b += level_bins(s.h[g], l);
  return b;
}
// number of bins before the lost bin
__host__ __device__ inline size_t sort_bins(const SysDev& s) { return bins_before(s, s.ngal, 0); }

// Host-side facts the launchers need to shape a multi-instance grid.
struct InstInfo {
  int64_t n;
  size_t grid_elems;  // grid elements cleared per step
  size_t dm_elems;  // density-maximum histogram (0: no galaxy uses it)
  bool fix;         // fixed-point mass assignment (the same for every instance of a launch)
};

struct Span {
  int ninst;
  int start[kMaxInst + 1];
};

int force_blocks(int64_t n);

template <typename T>
sbx_status launch_zero(T* p, size_t n, hipStream_t s);

// Zero every grid of every instance.
template <typename T>
sbx_status launch_zero_grids(const InstDev<T>* inst, const std::vector<InstInfo>& info, hipStream_t s);

// Zero the grids and compute the centres from the sums the last moving force
// pass left in com_partial, in one launch (valid when no instance uses
// density centring and the sums are current).
template <typename T>
sbx_status launch_zero_and_centres(const InstDev<T>* inst, const std::vector<InstInfo>& info,
                                   hipStream_t s);

// Loss test at the current positions and centre-of-mass sums (pre_partial),
// then the centres; with from_com the centres come from the sums the last
// moving force pass left in com_partial instead (no particle pass).
// Galaxies centred on their density maximum move from their current centre
// (the centres array) when density is set, and keep it otherwise.
template <typename T>
sbx_status launch_centres(const InstDev<T>* inst, const int* cur, const std::vector<InstInfo>& info,
                          bool from_com, hipStream_t s, bool density = true);

template <typename T>
sbx_status launch_deposit(const InstDev<T>* inst, const int* cur, const std::vector<InstInfo>& info,
                          hipStream_t s);

// mode bits: 1 = move (kick + drift + loss test; centre-of-mass sums of the
// new positions into com_partial), 2 = write acc/pot, 4 = diagnostics record
// into diag_out.
template <typename T>
sbx_status launch_force(const InstDev<T>* inst, const int* cur, const std::vector<InstInfo>& info,
                        int mode, hipStream_t s);

// Counting sort of every instance's particles by the cell of their finest
// grid (relative to their own galaxy) from set cur to set cur^1, then flips
// cur.  counts: the shared count buffer (sum of bins + 1 over instances),
// tmp: scan_tmp_elems(total counts).
template <typename T>
sbx_status launch_sort(const InstDev<T>* inst, int* cur, const std::vector<InstInfo>& info,
                       uint32_t* counts, size_t total_counts, uint32_t* tmp, hipStream_t s);

// single-instance helpers
template <typename T>
sbx_status launch_indices(const InstDev<T>* inst, const int* cur, int64_t n, int galaxy, int level,
                          int32_t* idx, int8_t* cls, hipStream_t s);

// Reverse mode of a leapfrog segment (single instance, fixed centres).
// init: loss (one double) and seeds of the adjoints; step: one reverse cycle
// at the positions in the live set with the forward fields in the grids,
// adjoint sources scattered into B; gather: mass gradient from the adjoint
// potentials P.  `out` marks the particles that sat out the cycle (lost at
// its start): their adjoints pass through unchanged and they gather nothing.
template <typename T>
sbx_status launch_adj_init(const InstDev<T>* inst, const int* cur, int64_t n, int sel_comp,
                           int sel_gal, double* lx, double* lv, double* gm, double* partial,
                           double* loss, hipStream_t s);
template <typename T>
sbx_status launch_adj_step(const InstDev<T>* inst, const int* cur, int64_t n, const GridsDev<T>& B,
                           const uint8_t* out, double* lx, double* lv, hipStream_t s);
template <typename T>
sbx_status launch_adj_gather(const InstDev<T>* inst, const int* cur, int64_t n, const GridsDev<T>& P,
                             const uint8_t* out, double* gm, hipStream_t s);

sbx_status launch_iota(int32_t* id, int64_t n, hipStream_t s);

// Bits of the largest of n non-negative masses into *out (device).
template <typename T>
sbx_status launch_mass_max(const T* m, int64_t n, unsigned long long* out, hipStream_t s);

// Device-side check of particle inputs (device arrays, host layout): the
// lowest bad index goes to *bad (device, preset to all ones by the caller).
sbx_status launch_validate_particles(const double* x, const double* v, const double* m,
                                     const int8_t* comp, const int8_t* gal, int64_t n, int ngal,
                                     unsigned long long* bad, hipStream_t s);

// As launch_validate_particles for structure-of-arrays inputs in precision
// T (x[k * n + i], v likewise).
template <typename T>
sbx_status launch_validate_soa(const T* x, const T* v, const T* m, const int8_t* comp,
                               const int8_t* gal, int64_t n, int ngal, unsigned long long* bad,
                               hipStream_t s);

// dst[id[i] * width + w] = src[i * width + w]
template <typename A>
sbx_status launch_unpermute(const A* src, const int32_t* id, A* dst, int64_t n, int width,
                            hipStream_t s);

template <typename T>
sbx_status launch_convert_in(const double* src, T* dst, size_t n, hipStream_t s);
template <typename T>
sbx_status launch_convert_out(const T* src, double* dst, size_t n, hipStream_t s);

// split host n*3 row-major doubles (already on device) into 3 SoA arrays of T
template <typename T>
sbx_status launch_split3(const double* src, T* x0, T* x1, T* x2, int64_t n, hipStream_t s);
template <typename T>
sbx_status launch_join3(const T* x0, const T* x1, const T* x2, double* dst, int64_t n,
                        hipStream_t s);

}  // namespace sbx
