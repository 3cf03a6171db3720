// Batched isolated-boundary Poisson solver on gfx950 (host interface).
//
// One solve turns an N^3 grid of cell masses into the field of Eq. 1 by the
// doubled-grid convolution of Eqs. 3-5: the (2N)^3 work grid is never formed.
// Five passes, each a batch of 1D FFTs of length L = 2N held in LDS:
//   fwd_x : rho[z][y][x]   (x < N)      -> X[kx][z][y]  (kx <= N, real-to-complex)
//   fwd_y : X[kx][z][y]    (y < N)      -> C[kx][ky][z] (ky < 2N)
//   zpass : C[kx][ky][z]   (z < N)      -> forward z, times Hhat, inverse z, keep z < N
//   inv_y : C[kx][ky][z]                -> X[kx][z][y]  (keep y < N)
//   inv_x : X[kx][z][y]    (kx <= N)    -> phi[z][y][x] (complex-to-real, keep x < N)
// Zero halves of the padded inputs are never read, unused halves of the
// outputs never written.  Hhat (real, even per axis) is stored on (N+1)^3.
#pragma once

#include "common.h"

namespace sbx {

template <typename T>
struct SolveDesc {
  const T* rho;   // N^3 cell masses
  T* phi;         // N^3 output (may alias rho)
  C2<T>* X;       // (N+1) * N * N
  C2<T>* C;       // (N+1) * 2N * N
  const T* H;     // (N+1)^3 transformed Green's function, scaled by G/(2N)^3
};

// Up to kMaxBatch solves of one grid size per launch; passed by value as a
// kernel argument (block-uniform index, read through scalar loads).
constexpr int kMaxBatch = 40;
template <typename T>
struct SolveBatch {
  SolveDesc<T> d[kMaxBatch];
};

// Per-precision, per-length twiddle tables (device), built once per device.
template <typename T>
const C2<T>* twiddles(int L, hipStream_t s);

// Workspace sizes in elements of C2<T>.
inline size_t x_elems(int N) { return (size_t)(N + 1) * N * N; }
inline size_t c_elems(int N) { return (size_t)(N + 1) * 2 * N * N; }
inline size_t h_elems(int N) { return (size_t)(N + 1) * (N + 1) * (N + 1); }

// Launch the five passes for the first `nsolves` (<= kMaxBatch) descriptors
// of one grid size N.  Returns SBX_OK or an error status.
template <typename T>
sbx_status solve_batch(int N, int nsolves, const SolveBatch<T>& b, hipStream_t s,
                       Recorder* rec = nullptr);

// Build the transformed Green's function for geometry (N, l, lz) into H
// ((N+1)^3 elements of T): FP64 H of Eq. 2 mirrored by Eq. 5, FP64 3D FFT,
// scaled by G/(2N)^3, folded.  rel_imag (host) receives max|Im|/max|Re|.
template <typename T>
sbx_status build_green(int N, double l, double lz, double G, int h0_mode, T* H, double* rel_imag,
                       hipStream_t s);

}  // namespace sbx
