// Batched isolated-boundary Poisson solver on gfx950 (host interface).
//
// One solve turns an N^3 grid of cell masses into the field of Eq. 1 by the
// doubled-grid convolution of Eqs. 3-5: the (2N)^3 work grid is never formed.
// Five passes, each a batch of 1D FFTs of length L = 2N held in LDS:
//   fwd_x : rho[z][y][x]   (x < N)      -> X[kx][z][y]  (kx <= N, real-to-complex)
//   fwd_y : X[kx][z][y]    (y < N)      -> C[kx][ky][z] (ky < 2N)
//   zpass : C[kx][ky][z]   (z < N)      -> forward z, times Hhat, inverse z, keep z < N,
//                                          stored as D[kx][z][ky]
//   inv_y : D[kx][z][ky]                -> E[z][y][kx]  (keep y < N; E reuses X)
//   inv_x : E[z][y][kx]    (kx <= N)    -> phi[z][y][x] (complex-to-real, keep x < N)
// Every pass reads whole lines (contiguous); the transposes are done on the
// write side, through LDS, in runs of at least 128 bytes.
// Where a z plane's half spectrum fits in LDS (32 <= N <= 64; at N = 128
// half of it, in FP32 and FP64) the same solve can run in three passes: plane forward (x and y of
// one plane in one block) -> P[z][kx][ky'] (in C; ky' = m for ky = 2m,
// N + m for 2m + 1), the z pass on that layout -> D, plane inverse (inverse
// y and x of one plane) -> phi.  At N = 128 the plane passes can run as
// two blocks per plane, each in half the LDS (two such blocks per CU in
// FP32, one in FP64, whose whole plane does not fit): the forward one for
// the even and one for the odd kx columns, the inverse one for the even
// and one for the odd rows y.  The tuner times both forms (and for the
// inverse, whole or half planes) and keeps the faster per precision, grid
// size and solve count.
// Zero halves of the padded inputs are never read, unused halves of the
// outputs never written.  Hhat (real, even per axis) is stored on (N+1)^3.
//
// Every pass is one persistent launch over all solves of one grid size:
// blocks pull (solve, tile) work items from a counter.  The size groups of a
// plan are independent and run concurrently, each on a stream of its own
// forked from and joined back to the caller's stream (concurrent branches
// when the caller captures a graph).  Line schedule (radix split), block
// size and grid size of each pass are chosen by timing the candidates the
// first time a precision, grid size and solve count is planned.
#pragma once

#include <vector>

#include "common.h"

namespace sbx {

template <typename T>
struct SolveDesc {
  const T* rho;   // N^3 cell masses
  const T* rho2;  // null, or N^3 cell masses added to rho (the summed grids)
  T* phi;         // N^3 output (may alias rho)
  C2<T>* X;       // (N+1) * N * N, also E: N * N rows of N + kEPad
  C2<T>* C;       // (N+1) * 2N * N
  C2<T>* D;       // (N+1) * N * 2N
  const T* H;     // (N+1)^3 transformed Green's function, scaled by G/(2N)^3
  int N;
};

constexpr int kPasses = 5;

// Launch shape of one pass.
struct PassShape {
  int nt;     // threads per block
  int grid;   // persistent blocks (0: one block per tile)
  int v = 0;  // values per thread of a line (16 or 32; 0: the length's default)
};

constexpr int kMaxGroups = 6;  // distinct grid sizes 8..256

// Solves of one grid size inside a plan.
struct SolveGroup {
  int first = 0, count = 0, N = 0;
  int form = 5;                      // 5 line passes, or 3 plane-fused passes
  const void* tw[kPasses] = {};      // twiddle table of each pass's lines (2N; N for the plane passes)
  const void* twist = nullptr;       // plane form: exp(-2 pi i n / 2N), n < N
  PassShape shape[kPasses] = {};
};

template <typename T>
struct SolvePlan {
  int nsolves = 0;
  std::vector<SolveDesc<T>> host;    // grouped by grid size
  SolveDesc<T>* d_solves = nullptr;
  int* d_counter = nullptr;          // kPasses * kMaxGroups work counters
  int ngroups = 0;
  SolveGroup groups[kMaxGroups];
  // with several groups: streams of groups 1.. (group 0 runs on the
  // caller's stream) and the fork and join events
  hipStream_t side[kMaxGroups] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxGroups] = {};
};

// Workspace sizes in elements of C2<T>.
// E rows (kx = 0..N) are padded to N + 16 entries so that every row starts
// on a 128-byte boundary; X (the forward layout) fits in the same space.
constexpr int kEPad = 16;
inline size_t x_elems(int N) { return (size_t)N * N * (N + kEPad); }
inline size_t c_elems(int N) { return (size_t)(N + 1) * 2 * N * N; }
// C and D of one solve, back to back (D = C + c_elems(N))
inline size_t cd_elems(int N) { return 2 * c_elems(N); }
inline size_t h_elems(int N) { return (size_t)(N + 1) * (N + 1) * (N + 1); }

// Prepare a plan for the given solves (device tables, twiddles, launch
// shapes from the tuning cache; tunes on the plan's own buffers when the mix
// of grid sizes is new -- rho/phi/X/C are then overwritten with zeros).
template <typename T>
sbx_status plan_create(SolvePlan<T>& plan, const SolveDesc<T>* descs, int n, hipStream_t s);

// Run all solves of the plan (five launches per size group; each pass
// clears the work counter of the pass before it, so the counters are zero
// between runs).  With several size groups the groups run on concurrent
// streams between a fork and a join on s; phase marks are then all taken
// at the join.
template <typename T>
sbx_status plan_run(const SolvePlan<T>& plan, hipStream_t s, Recorder* rec = nullptr);

// One pass (0..4) of one size group, for callers that schedule the groups
// themselves (e.g. as concurrent branches of a graph).  Clears the work
// counter of the previous pass of the group: run the passes of a group in
// order 0..4, each after the one before it has finished.
template <typename T>
sbx_status plan_run_pass(const SolvePlan<T>& plan, int pass, int group, hipStream_t s);

template <typename T>
void plan_destroy(SolvePlan<T>& plan);

// Make (once per device, precision and length; allocates) the twiddle table
// of the solves of N^3 grids.
template <typename T>
sbx_status prepare_twiddles(int N, hipStream_t s);

// The five passes of nsolves solves of N^3 grids whose descriptors are
// already in device memory, with the tuned launch shapes of (T, N, nsolves)
// when cached and default shapes otherwise.  Launches only: allocates
// nothing and waits for nothing (the twiddle table must exist).  d_counter:
// kPasses work counters, zero on entry, left nonzero.
template <typename T>
sbx_status run_solves_noalloc(const SolveDesc<T>* d_solves, int nsolves, int N, int* d_counter,
                              hipStream_t s);

// Pin the line schedule of plans tuned from now on to v values per thread
// (16 or 32, where a line length has both; 0: time both).  Process-wide.
sbx_status set_fft_schedule(int v);

// Pin the form of plans tuned from now on: 3 (plane-fused passes, where a
// plane fits in LDS), 5 (five line passes) or 0 (time both).  Process-wide.
sbx_status set_fft_form(int f);
// Pin the block size of the plane passes tuned from now on: 256, 512, 1024
// or 0 (time all).  Process-wide.
sbx_status set_plane_threads(int nt);

// Whether launch shapes for this precision and mix of grid sizes are cached.
bool tuning_cached(int esz, std::vector<int> mix);

// Tuned launch shapes of every mix planned so far, as text (one line per
// pass and mix), for reports.
std::string tuning_report();

// Build the transformed Green's function for geometry (N, l, lz) into H
// ((N+1)^3 elements of T): FP64 H of Eq. 2 mirrored by Eq. 5, FP64 3D FFT,
// scaled by G/(2N)^3, folded.  rel_imag (host) receives max|Im|/max|Re|.
template <typename T>
sbx_status build_green(int N, double l, double lz, double G, int h0_mode, T* H, double* rel_imag,
                       hipStream_t s);

}  // namespace sbx
