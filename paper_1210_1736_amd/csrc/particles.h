// Particle-side kernels of the nested-grid PM step (host interface).
#pragma once

#include "common.h"

namespace sbx {

constexpr int kMaxGal = 4;       // galaxies per context
constexpr int kSlots = 5;        // grids per 3-level galaxy
constexpr int kNComp = 8;        // particle component ids
// diagnostics record: per component [ekin, epot, Lx, Ly, Lz, count],
// disc [sum vR, sum vR^2, sum vz, sum vz^2, count], lost count
constexpr int kDiagComp = 6;
constexpr int kDiagDisc = kNComp * kDiagComp;
constexpr int kDiagLost = kDiagDisc + 5;
constexpr int kNDiag = kDiagLost + 1;
constexpr int kPreVals = kMaxGal * 4;  // per galaxy [m, m x, m y, m z]
constexpr int kRedBlocks = 1024;       // grid of the loss-test / centre-of-mass pass
constexpr int kForceBlocksMax = 4096;  // grid cap of the force pass (partial rows)

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
  int centring;  // 0 fixed, 1 centre of mass
  LevelDev lv[3];
  double centre[3];   // fixed centre (inner/middle levels, or the single grid)
  double outer_c[3];  // centre of the global grid (3 levels)
};

struct SysDev {
  int ngal;
  int taylor;
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
// (global, outer), 4: grids 4+5 (global, all).  1 level -> slot 0 only.
template <typename T>
struct GridsDev {
  T* g[kMaxGal][kSlots];
};

template <typename T>
sbx_status launch_zero(T* p, size_t n, hipStream_t s);

// Loss test at the current positions plus centre-of-mass partial sums
// (kRedBlocks rows of kPreVals into partial), then the centres.
template <typename T>
sbx_status launch_pre(const PartDev<T>& p, const SysDev& sys, double* partial, double* centres,
                      hipStream_t s);

// Centres from centre-of-mass partial sums (rows x kPreVals) written by the
// previous moving force pass; `sums` receives the kPreVals column totals.
sbx_status launch_centres(const double* partial, int rows, const SysDev& sys, double* sums,
                          double* centres, hipStream_t s);

int force_blocks(int64_t n);

// Counting sort of the particles by the cell of their finest grid (relative
// to their own galaxy): src -> dst.  key: n uint32; count: bins + 1 uint32
// (bins = ngal * 3 * N^3); tmp: scan_tmp_elems(bins + 1).
template <typename T>
sbx_status launch_sort(const PartDev<T>& src, const PartDev<T>& dst, const SysDev& sys,
                       const double* centres, uint32_t* key, uint32_t* count, size_t bins,
                       uint32_t* tmp, hipStream_t s);

sbx_status launch_iota(int32_t* id, int64_t n, hipStream_t s);

// dst[id[i] * width + w] = src[i * width + w]
template <typename A>
sbx_status launch_unpermute(const A* src, const int32_t* id, A* dst, int64_t n, int width,
                            hipStream_t s);

template <typename T>
sbx_status launch_deposit(const PartDev<T>& p, const SysDev& sys, const double* centres,
                          const GridsDev<T>& grids, hipStream_t s);

// mode bits: 1 = move (kick + drift + loss test; centre-of-mass partial sums
// of the new positions into com_partial, force_blocks(n) rows of kPreVals),
// 2 = write acc/pot (float64, acc n*3 row-major, pot = physical phi),
// 4 = diagnostics record into diag_out (kNDiag doubles) via partial
// (force_blocks(n) rows of kNDiag).
template <typename T>
sbx_status launch_force(const PartDev<T>& p, const SysDev& sys, const double* centres,
                        const GridsDev<T>& fields, double dt, int mode, double* acc, double* pot,
                        double* partial, double* diag_out, double* com_partial, hipStream_t s);

template <typename T>
sbx_status launch_indices(const PartDev<T>& p, const SysDev& sys, const double* centres, int galaxy,
                          int level, int32_t* idx, int8_t* cls, hipStream_t s);

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
