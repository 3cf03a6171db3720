// Batched pruned 3D FFT convolution with the isolated-boundary Green's
// function (Eqs. 3-5 of the method) and the FP64 Green's-table build.
//
// Each block holds W lines of length L = 2N in LDS and runs a Stockham
// autosort FFT on them: a first pass of radix 16 (radix 32 for L = 512) with
// one DFT in registers per thread, then the remaining radix (2, 4, 8 or 16)
// with twiddles from a table.  Global loads and stores are arranged so that consecutive threads
// touch consecutive addresses: along the line when the line is contiguous,
// across the W lines of a tile when it is strided.
#include <algorithm>
#include <array>
#include <cstring>
#include <atomic>
#include <mutex>
#include <type_traits>

#include "fft.h"

namespace sbx {

__device__ __forceinline__ int pad(int e) { return e + (e >> 4); }

// ------------------------------------------------------------- Stockham ---
// A line of length L is transformed by TL = L/VPT threads of one wavefront
// (64/TL lines per wave), each holding VPT values (16, or 32 for L = 512 in
// FP32), so the exchanges between the passes go through LDS with wave-level
// ordering only.  Passes: radix VPT (stride 1), then radix L/VPT with stride
// VPT (VPT/R butterflies of radix R per thread); in FP64 at L = 512 the
// second pass is radix 16 and a radix-2 pass with stride 256 follows (32
// complex doubles per thread would not leave room for the rest).
//
// Forward pass p (decimation in time, Stockham autosort): butterfly j reads
// positions j + r*L/R, multiplies by twiddles, takes the R-point DFT and
// writes positions (j - k) R + k + r NS, k = j mod NS.  The inverse
// transform runs the conjugate transposes of the same passes in reverse
// order (gather from the output positions, inverse DFT, conjugate twiddles,
// scatter to the input positions).  The last forward pass reads and writes
// the same positions, which is what lets the z pass apply the Green's
// function and the first inverse pass in registers.
template <typename T, int L, int V>
struct Line {
  static constexpr int VPT = V;
  static constexpr int TL = L / VPT;
  static constexpr int NP = L == 16 ? 1 : (L / VPT <= 16 ? 2 : 3);
  template <int p>
  static constexpr int R = p == 0 ? VPT : (p == 1 ? (L / VPT <= 16 ? L / VPT : 16) : 2);
  template <int p>
  static constexpr int NS = p == 0 ? 1 : (p == 1 ? VPT : 16 * VPT);
  template <int p>
  static constexpr int TW = p == 2 ? 15 * VPT : 0;  // offset of the pass in the twiddle table
};

// The schedule of a line length unless the autotuner picks the other one:
// 32 values per thread for L = 512 in FP32, else 16.  In FP32, lines of
// L >= 128 have both (16: radix 16 then L/16 (then 2); 32: radix 32 then
// L/32), and the tuner times both.
template <typename T, int L>
constexpr int kDefV = (L == 512 && sizeof(T) == 4) ? 32 : 16;
template <typename T, int L>
constexpr bool kTwoV = sizeof(T) == 4 && L >= 128;

// Order the LDS accesses of one wavefront (they execute in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int L, int V, int p>
__device__ __forceinline__ int pos_in(int j, int r) {
  return j + r * (L / Line<T, L, V>::template R<p>);
}
template <typename T, int L, int V, int p>
__device__ __forceinline__ int pos_out(int j, int r) {
  constexpr int NS = Line<T, L, V>::template NS<p>, R = Line<T, L, V>::template R<p>;
  const int k = j & (NS - 1);
  return (j - k) * R + k + r * NS;
}

template <typename T, int L, int V, int p>
__device__ __forceinline__ void fwd_bfly(C2<T>* v, int t, const C2<T>* __restrict__ tw) {
  using F = Line<T, L, V>;
  constexpr int R = F::template R<p>, NS = F::template NS<p>, BPT = F::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    if constexpr (NS > 1) {
      const int k = (t + b * F::TL) & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r)
        v[b * R + r] = cmul(v[b * R + r], tw[F::template TW<p> + (r - 1) * NS + k]);
    }
    dftR<R, false>(v + b * R);
  }
}

template <typename T, int L, int V, int p>
__device__ __forceinline__ void inv_bfly(C2<T>* v, int t, const C2<T>* __restrict__ tw) {
  using F = Line<T, L, V>;
  constexpr int R = F::template R<p>, NS = F::template NS<p>, BPT = F::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    dftR<R, true>(v + b * R);
    if constexpr (NS > 1) {
      const int k = (t + b * F::TL) & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r)
        v[b * R + r] = cmul(v[b * R + r], conjc(tw[F::template TW<p> + (r - 1) * NS + k]));
    }
  }
}

// LDS gathers and scatters of one line (padded by one element per 16).
// ZHI: the upper half of the line's input is zero (padded input).
template <typename T, int L, int V, int p, bool ZHI>
__device__ __forceinline__ void gather_in(const C2<T>* s, int t, C2<T>* v) {
  constexpr int R = Line<T, L, V>::template R<p>, BPT = Line<T, L, V>::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r)
      v[b * R + r] = (ZHI && r >= R / 2) ? C2<T>{(T)0, (T)0}
                                         : s[pad(pos_in<T, L, V, p>(t + b * Line<T, L, V>::TL, r))];
}
// HALF: only positions below L/2 are kept (cropped output).
template <typename T, int L, int V, int p, bool HALF>
__device__ __forceinline__ void scatter_in(C2<T>* s, int t, const C2<T>* v) {
  constexpr int R = Line<T, L, V>::template R<p>, BPT = Line<T, L, V>::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (!HALF || r < R / 2) s[pad(pos_in<T, L, V, p>(t + b * Line<T, L, V>::TL, r))] = v[b * R + r];
}
template <typename T, int L, int V, int p>
__device__ __forceinline__ void gather_out(const C2<T>* s, int t, C2<T>* v) {
  constexpr int R = Line<T, L, V>::template R<p>, BPT = Line<T, L, V>::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = s[pad(pos_out<T, L, V, p>(t + b * Line<T, L, V>::TL, r))];
}
template <typename T, int L, int V, int p>
__device__ __forceinline__ void scatter_out(C2<T>* s, int t, const C2<T>* v) {
  constexpr int R = Line<T, L, V>::template R<p>, BPT = Line<T, L, V>::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) s[pad(pos_out<T, L, V, p>(t + b * Line<T, L, V>::TL, r))] = v[b * R + r];
}

// Forward passes PS..NP-1 on an LDS line, in place; v holds the inputs of
// pass PS on entry (already gathered) and the last pass's outputs (natural
// order, positions j + r L/R) on exit, also written to LDS when STORE.
template <typename T, int L, int V, int PS, bool STORE>
__device__ __forceinline__ void fwd_from(C2<T>* s, int t, C2<T>* v, const C2<T>* __restrict__ tw) {
  constexpr int NP = Line<T, L, V>::NP;
  fwd_bfly<T, L, V, PS>(v, t, tw);
  if constexpr (PS + 1 < NP) {
    scatter_out<T, L, V, PS>(s, t, v);
    wave_sync();
    gather_in<T, L, V, PS + 1, false>(s, t, v);
    wave_sync();
    fwd_from<T, L, V, PS + 1, STORE>(s, t, v, tw);
  } else if constexpr (STORE) {
    scatter_out<T, L, V, PS>(s, t, v);
  }
}

// Inverse passes PE..0 (conjugate transposes, reverse order); v holds the
// inputs of pass PE (gathered at its output positions) on entry and the
// natural-order results of pass 0 (positions t + r TL) on exit.
template <typename T, int L, int V, int PE>
__device__ __forceinline__ void inv_down(C2<T>* s, int t, C2<T>* v, const C2<T>* __restrict__ tw) {
  inv_bfly<T, L, V, PE>(v, t, tw);
  if constexpr (PE > 0) {
    scatter_in<T, L, V, PE, false>(s, t, v);
    wave_sync();
    gather_out<T, L, V, PE - 1>(s, t, v);
    wave_sync();
    inv_down<T, L, V, PE - 1>(s, t, v, tw);
  }
}

// Full forward transform of a line held in LDS in natural order (in place).
template <typename T, int L, int V>
__device__ __forceinline__ void line_fwd_lds(C2<T>* s, int t, const C2<T>* __restrict__ tw) {
  C2<T> v[Line<T, L, V>::VPT];
  gather_in<T, L, V, 0, false>(s, t, v);
  wave_sync();
  fwd_from<T, L, V, 0, true>(s, t, v, tw);
  wave_sync();
}

template <typename T>
__global__ void k_twiddle(C2<T>* tw, int R, int NS) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (R - 1) * NS) return;
  const int r = 1 + i / NS, k = i % NS;
  double s, c;
  sincospi(2.0 * (double)(k * r) / (double)(NS * R), &s, &c);
  tw[i] = C2<T>{(T)c, (T)(-s)};
}

// Twiddle table for length L: for every pass after the first, at the
// pass's offset, entries (r-1)*NS + k = exp(-2 pi i k r / (NS R)),
// r = 1..R-1, k = 0..NS-1.
template <typename T, int L, int V, int p>
static int tw_fill(C2<T>* tw, hipStream_t st) {
  using F = Line<T, L, V>;
  if constexpr (p >= F::NP) {
    return F::template TW<p - 1> + (F::template R<p - 1> - 1) * F::template NS<p - 1>;
  } else {
    constexpr int R = F::template R<p>, NS = F::template NS<p>, n = (R - 1) * NS;
    if (tw) hipLaunchKernelGGL(k_twiddle<T>, dim3((n + 255) / 256), dim3(256), 0, st,
                               tw + F::template TW<p>, R, NS);
    return tw_fill<T, L, V, p + 1>(tw, st);
  }
}

template <typename T, int L>
static int tw_make_l(int V, C2<T>* tw, hipStream_t st) {
  if constexpr (kTwoV<T, L>) {
    if (V == 32) return tw_fill<T, L, 32, 1>(tw, st);
    if (V == 16) return tw_fill<T, L, 16, 1>(tw, st);
  }
  return tw_fill<T, L, kDefV<T, L>, 1>(tw, st);
}

template <typename T>
static int tw_make(int L, int V, C2<T>* tw, hipStream_t st) {
  switch (L) {
    case 16: return 1;
    case 32: return tw_make_l<T, 32>(V, tw, st);
    case 64: return tw_make_l<T, 64>(V, tw, st);
    case 128: return tw_make_l<T, 128>(V, tw, st);
    case 256: return tw_make_l<T, 256>(V, tw, st);
    default: return tw_make_l<T, 512>(V, tw, st);
  }
}

// Schedule actually used for values per thread v of a line length (0 or an
// unavailable value: the default one).
template <typename T>
static int eff_v(int L, int v) {
  const bool two = sizeof(T) == 4 && L >= 128;
  const int def = (L == 512 && sizeof(T) == 4) ? 32 : 16;
  return two && (v == 16 || v == 32) ? v : def;
}

// Twiddle tables are made once per (device, precision, length, schedule)
// and kept for the life of the process.  With create = false a missing
// table is not made (nothing is allocated) and null is returned.
template <typename T>
const C2<T>* twiddles(int L, int v, hipStream_t st, bool create = true) {
  static std::mutex mu;
  static C2<T>* cache[64][10][2] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  const int V = eff_v<T>(L, v), vi = V == 32 ? 1 : 0;
  std::lock_guard<std::mutex> g(mu);
  if (cache[dev][lg][vi] || !create) return cache[dev][lg][vi];
  C2<T>* p = nullptr;
  if (hipMalloc(&p, sizeof(C2<T>) * tw_make<T>(L, V, nullptr, st)) != hipSuccess) return nullptr;
  tw_make<T>(L, V, p, st);
  if (hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(p);
    return nullptr;
  }
  cache[dev][lg][vi] = p;
  return p;
}

template const C2<float>* twiddles<float>(int, int, hipStream_t, bool);
template const C2<double>* twiddles<double>(int, int, hipStream_t, bool);

// ------------------------------------------------------------ tile shape ---
// A block of NT threads covers WT = NT/TL lines at a time.  The z pass takes
// W = WT lines per tile (each wave its own lines, no block barrier).  The x
// and y passes, whose other side is strided across lines, take at least
// 128 bytes of lines per tile (the block loops over them in rounds) within
// the LDS budget; a tile's lines are staged in LDS for the strided side.
constexpr int kLdsCap = 81920;  // two blocks per compute unit

template <typename T, int L, int V, int NT, int PASS>
struct TC {
  static constexpr int N = L / 2;
  static constexpr int TL = Line<T, L, V>::TL;
  static constexpr int P = L + L / 16 + 1;  // LDS pitch of one line
  static constexpr int LB = P * (int)sizeof(C2<T>);
  static constexpr int WT = NT / TL;
  static constexpr int WC = 128 / (int)sizeof(C2<T>);
  static constexpr int fitw(int w) { return (w > 1 && w * LB > kLdsCap) ? fitw(w / 2) : w; }
  static constexpr int fitw2(int w) { return (w > 2 && (w / 2) * LB > kLdsCap) ? fitw2(w / 2) : w; }
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int mn(int a, int b) { return a < b ? a : b; }
  // W: grid rows per tile.  fwd_x packs two real rows into one complex line
  // (W/2 lines, at least 128 bytes per stored run); the z pass takes one
  // round of lines; inv_x takes one round of complex lines, each two real
  // rows (2 W rows per tile); fwd_y and inv_y at least 128 bytes per run.
  static constexpr int W = PASS == 0   ? fitw2(mn(N, mx(2 * WT, WC)))
                         : (PASS == 2 || PASS == 5) ? mn(WT, L)
                         : PASS == 4 ? mn(WT, N / 2)
                                     : fitw(mn(N, mx(WT, WC)));
  static constexpr int LINES = PASS == 0 ? W / 2 : W;  // lines held in LDS
  static constexpr bool fits = LINES * LB <= kLdsCap;
  static constexpr int LDS = fits ? LINES * P : 1;     // elements of C2<T>
  static constexpr int ROUNDS = (LINES + WT - 1) / WT;
};

// tiles of each pass for one solve of line length L (the inverse y pass
// tiles kx = 0..N, the last tile partly)
template <typename T, int L, int V, int NT>
__host__ __device__ constexpr int tiles_of(int pass) {
  constexpr int N = L / 2;
  return pass == 0 ? N * (N / TC<T, L, V, NT, 0>::W)
       : pass == 1 ? (N + 1) * (N / TC<T, L, V, NT, 1>::W)
       : (pass == 2 || pass == 5) ? (N + 1) * (L / TC<T, L, V, NT, 2>::W)
       : pass == 3 ? N * ((N + TC<T, L, V, NT, 3>::W) / TC<T, L, V, NT, 3>::W)
                   : N * (N / (2 * TC<T, L, V, NT, 4>::W));
}

template <typename T, int L, int V, int NT, int PASS>
__host__ __device__ constexpr bool shape_fits() {
  return TC<T, L, V, NT, PASS>::fits;
}

// Complex values through global-memory views (member-wise: the struct's
// assignment works on generic pointers only).
template <typename T>
__device__ __forceinline__ C2<T> gld(gp<const C2<T>> p) {
  return C2<T>{p->re, p->im};
}
template <typename T>
__device__ __forceinline__ void gst(gp<C2<T>> p, const C2<T>& v) {
  p->re = v.re;
  p->im = v.im;
}

// ------------------------------------------------------------ the passes ---
// Each pass reads its input lines once: those loads are non-temporal, so
// they do not displace the lines the pass is writing (the next pass's
// input) from the caches.
// fwd_x: tile = W consecutive y at one z; real rows x < N taken two at a
// time as the real and imaginary parts of one complex line (straight into
// registers); after the transform the two spectra are separated by
// Hermitian symmetry, X_a = (Z + conj Z(-k)) / 2, X_b = -i (Z - conj Z(-k)) / 2,
// and stored as X[kx][z][y] (kx <= N) across rows.
template <typename T, int L, int V, int NT>
__device__ __forceinline__ void tile_fwd_x(const SolveDesc<T>& d, int tile, C2<T>* s,
                                           const C2<T>* __restrict__ tw) {
  using K = TC<T, L, V, NT, 0>;
  constexpr int N = K::N, W = K::W, P = K::P, TL = K::TL, WL = K::LINES;
  const int tid = threadIdx.x, t = tid % TL;
  const int z = tile / (N / W), y0 = (tile % (N / W)) * W;
#pragma unroll 1
  for (int u = 0; u < K::ROUNDS; ++u) {
    const int j = u * K::WT + tid / TL;
    if (j < WL) {
      const size_t row = ((size_t)z * N + y0 + 2 * j) * N;
      const gp<const T> __restrict__ a = glb(d.rho + row);
      const gp<const T> __restrict__ b = a + N;
      constexpr int VPT = Line<T, L, V>::VPT;
      C2<T> v[VPT];
#pragma unroll
      for (int r = 0; r < VPT; ++r)
        v[r] = r < VPT / 2 ? C2<T>{__builtin_nontemporal_load(&a[t + r * TL]), __builtin_nontemporal_load(&b[t + r * TL])} : C2<T>{(T)0, (T)0};
      if (d.rho2) {  // summed grids: the second source is added on the way in
        const gp<const T> __restrict__ a2 = glb(d.rho2 + row);
        const gp<const T> __restrict__ b2 = a2 + N;
#pragma unroll
        for (int r = 0; r < VPT / 2; ++r) {
          v[r].re += a2[t + r * TL];
          v[r].im += b2[t + r * TL];
        }
      }
      fwd_from<T, L, V, 0, true>(s + j * P, t, v, tw);
    }
  }
  __syncthreads();
  const gp<C2<T>> __restrict__ dst = glb(d.X + (size_t)z * N + y0);
  const T h = (T)0.5;
  for (int i = tid; i < W * (N + 1); i += NT) {
    const int e = i / W, w = i - e * W;
    const C2<T>* sl = s + (w >> 1) * P;
    const C2<T> Z = sl[pad(e)], R = sl[pad(e == 0 ? 0 : L - e)];
    gst(dst + (size_t)e * N * N + w, (w & 1) ? C2<T>{(Z.im + R.im) * h, (R.re - Z.re) * h}
                                            : C2<T>{(Z.re + R.re) * h, (Z.im - R.im) * h});
  }
}

// fwd_y: tile = W consecutive z at one kx; each line (y < N, contiguous) read
// straight into registers; output C[kx][ky][z] stored across lines.
template <typename T, int L, int V, int NT>
__device__ __forceinline__ void tile_fwd_y(const SolveDesc<T>& d, int tile, C2<T>* s,
                                           const C2<T>* __restrict__ tw) {
  using K = TC<T, L, V, NT, 1>;
  constexpr int N = K::N, W = K::W, P = K::P, TL = K::TL;
  const int tid = threadIdx.x, t = tid % TL;
  const int kx = tile / (N / W), z0 = (tile % (N / W)) * W;
#pragma unroll 1
  for (int u = 0; u < K::ROUNDS; ++u) {
    const int w = u * K::WT + tid / TL;
    if (w < W) {
      const gp<const C2<T>> __restrict__ src = glb(d.X + ((size_t)kx * N + z0 + w) * N);
      constexpr int VPT = Line<T, L, V>::VPT;
      C2<T> v[VPT];
#pragma unroll
      for (int r = 0; r < VPT; ++r) v[r] = r < VPT / 2 ? C2<T>{__builtin_nontemporal_load(&src[t + r * TL].re), __builtin_nontemporal_load(&src[t + r * TL].im)} : C2<T>{(T)0, (T)0};
      fwd_from<T, L, V, 0, true>(s + w * P, t, v, tw);
    }
  }
  __syncthreads();
  const gp<C2<T>> __restrict__ dst = glb(d.C + (size_t)kx * L * N + z0);
  for (int i = tid; i < W * L; i += NT) {
    const int e = i / W, w = i - e * W;
    gst(dst + (size_t)e * N + w, s[w * P + pad(e)]);
  }
}

// zpass: tile = W consecutive ky at one kx, one line per TL threads; forward
// z (input z < N) from global, times Hhat in registers, inverse z, keep
// z < N; stored transposed as D[kx][z][ky] through LDS.
// PLANE: the spectra of the plane-fused passes, P[kx][z][ky'] in and out
// (ky' = m for ky = 2m, N + m for ky = 2m + 1): a tile's W lines are W
// consecutive ky' at one kx, gathered along z through LDS in runs of W
// from one kx slab.
template <typename T, int L, int V, int NT, bool PLANE>
__device__ __forceinline__ void tile_zpass(const SolveDesc<T>& d, int tile, C2<T>* s,
                                           const C2<T>* __restrict__ tw) {
  using K = TC<T, L, V, NT, 2>;
  using F = Line<T, L, V>;
  constexpr int N = K::N, W = K::W, P = K::P, TL = K::TL, NP = F::NP;
  constexpr int RL = F::template R<NP - 1>, NBL = L / RL;
  const int tid = threadIdx.x, t = tid % TL, w = tid / TL;
  const int kx = tile / (L / W), ky0 = (tile % (L / W)) * W;
  if constexpr (PLANE) {
    const gp<const C2<T>> __restrict__ g = glb(d.C + (size_t)kx * N * L + ky0);
    for (int i = tid; i < W * N; i += NT) {
      const int z = i / W, ww = i - z * W;
      const gp<const C2<T>> e = g + (size_t)z * L + ww;
      s[ww * P + pad(z)] = C2<T>{__builtin_nontemporal_load(&e->re), __builtin_nontemporal_load(&e->im)};
    }
    __syncthreads();
  }
  if (w < W) {
    const int kyl = ky0 + w;
    // the frequency of line w along y
    const int ky = PLANE ? (kyl < N ? 2 * kyl : 2 * (kyl - N) + 1) : kyl;
    C2<T>* sl = s + w * P;
    C2<T> v[F::VPT];
    if constexpr (PLANE) {
#pragma unroll
      for (int r = 0; r < F::VPT; ++r) v[r] = r < F::VPT / 2 ? sl[pad(t + r * TL)] : C2<T>{(T)0, (T)0};
    } else {
      const gp<const C2<T>> __restrict__ g = glb(d.C + ((size_t)kx * L + ky) * N);
#pragma unroll
      for (int r = 0; r < F::VPT; ++r) v[r] = r < F::VPT / 2 ? C2<T>{__builtin_nontemporal_load(&g[t + r * TL].re), __builtin_nontemporal_load(&g[t + r * TL].im)} : C2<T>{(T)0, (T)0};
    }
    if constexpr (NP > 1) {
      fwd_bfly<T, L, V, 0>(v, t, tw);
      scatter_out<T, L, V, 0>(sl, t, v);
      wave_sync();
      gather_in<T, L, V, 1, false>(sl, t, v);
      wave_sync();
      if constexpr (NP > 2) {
        fwd_bfly<T, L, V, 1>(v, t, tw);
        scatter_out<T, L, V, 1>(sl, t, v);
        wave_sync();
        gather_in<T, L, V, 2, false>(sl, t, v);
        wave_sync();
      }
    }
    fwd_bfly<T, L, V, NP - 1>(v, t, tw);
    // Hhat at frequencies (kx, ky, e), e = j + r L/R of the last pass
    const gp<const T> __restrict__ H = glb(d.H + ((size_t)kx * (N + 1) + (ky <= N ? ky : L - ky)) * (N + 1));
#pragma unroll
    for (int b = 0; b < F::VPT / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int e = t + b * TL + r * NBL;
        v[b * RL + r] = cscale(v[b * RL + r], H[e <= N ? e : L - e]);
      }
    inv_down<T, L, V, NP - 1>(sl, t, v, tw);
    wave_sync();
#pragma unroll
    for (int r = 0; r < F::VPT / 2; ++r) sl[pad(t + r * TL)] = v[r];
  }
  __syncthreads();
  if constexpr (PLANE) {
    const gp<C2<T>> __restrict__ dst = glb(d.D + (size_t)kx * N * L + ky0);
    for (int i = tid; i < W * N; i += NT) {
      const int z = i / W, ww = i - z * W;
      gst(dst + (size_t)z * L + ww, s[ww * P + pad(z)]);
    }
  } else {
    const gp<C2<T>> __restrict__ dst = glb(d.D + (size_t)kx * N * L + ky0);
    for (int i = tid; i < W * N; i += NT) {
      const int z = i / W, ww = i - z * W;
      gst(dst + (size_t)z * L + ww, s[ww * P + pad(z)]);
    }
  }
}

// inv_y: tile = W consecutive kx (<= N) at one z; lines D[kx][z][0..2N)
// read straight into registers; output y < N stored transposed as
// E[z][y][kx] (in the X buffer, rows padded to N + kEPad) through LDS.
template <typename T, int L, int V, int NT>
__device__ __forceinline__ void tile_inv_y(const SolveDesc<T>& d, int tile, C2<T>* s,
                                           const C2<T>* __restrict__ tw) {
  using K = TC<T, L, V, NT, 3>;
  using F = Line<T, L, V>;
  constexpr int N = K::N, W = K::W, P = K::P, TL = K::TL, NP = F::NP;
  constexpr int RL = F::template R<NP - 1>, NBL = L / RL;
  constexpr int NKT = (N + W) / W;  // kx tiles
  const int tid = threadIdx.x, t = tid % TL;
  const int z = tile / NKT, kx0 = (tile % NKT) * W;
#pragma unroll 1
  for (int u = 0; u < K::ROUNDS; ++u) {
    const int w = u * K::WT + tid / TL;
    if (w < W && kx0 + w <= N) {
      const gp<const C2<T>> __restrict__ src = glb(d.D + ((size_t)(kx0 + w) * N + z) * L);
      C2<T>* sl = s + w * P;
      C2<T> v[F::VPT];
      // inputs of the first inverse pass: natural positions of the last pass
#pragma unroll
      for (int b = 0; b < F::VPT / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) v[b * RL + r] = C2<T>{__builtin_nontemporal_load(&src[t + b * TL + r * NBL].re), __builtin_nontemporal_load(&src[t + b * TL + r * NBL].im)};
      inv_down<T, L, V, NP - 1>(sl, t, v, tw);
      wave_sync();
#pragma unroll
      for (int r = 0; r < F::VPT / 2; ++r) sl[pad(t + r * TL)] = v[r];
    }
  }
  __syncthreads();
  const gp<C2<T>> __restrict__ dst = glb(d.X + (size_t)z * N * (N + kEPad) + kx0);
  for (int i = tid; i < W * N; i += NT) {
    const int y = i / W, w = i - y * W;
    if (kx0 + w <= N) gst(dst + (size_t)y * (N + kEPad) + w, s[w * P + pad(y)]);
  }
}

// inv_x: tile = 2W consecutive y at one z; the lines E[z][y][0..N] of two
// rows (each extended to 2N by Hermitian symmetry) are combined as A + iB
// into one complex line, read straight into registers; the inverse
// transform's real and imaginary parts are the two real output rows x < N.
// No block barrier.
template <typename T, int L, int V, int NT>
__device__ __forceinline__ void tile_inv_x(const SolveDesc<T>& d, int tile, C2<T>* s,
                                           const C2<T>* __restrict__ tw) {
  using K = TC<T, L, V, NT, 4>;
  using F = Line<T, L, V>;
  constexpr int N = K::N, W = K::W, P = K::P, TL = K::TL, NP = F::NP;
  constexpr int RL = F::template R<NP - 1>, NBL = L / RL;
  const int tid = threadIdx.x, t = tid % TL, j = tid / TL;
  const int z = tile / (N / (2 * W)), y0 = (tile % (N / (2 * W))) * 2 * W;
  if (j >= W) return;
  const gp<const C2<T>> __restrict__ A = glb(d.X + ((size_t)z * N + y0 + 2 * j) * (N + kEPad));
  const gp<const C2<T>> __restrict__ B = A + (N + kEPad);
  C2<T>* sl = s + j * P;
  C2<T> v[F::VPT];
#pragma unroll
  for (int b = 0; b < F::VPT / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int e = t + b * TL + r * NBL;
      if (e <= N) {
        const C2<T> a = gld(A + e), q = gld(B + e);
        v[b * RL + r] = C2<T>{a.re - q.im, a.im + q.re};
      } else {
        const C2<T> a = gld(A + (L - e)), q = gld(B + (L - e));
        v[b * RL + r] = C2<T>{a.re + q.im, q.re - a.im};
      }
    }
  inv_down<T, L, V, NP - 1>(sl, t, v, tw);
  const gp<T> __restrict__ da = glb(d.phi + ((size_t)z * N + y0 + 2 * j) * N);
  const gp<T> __restrict__ db = da + N;
#pragma unroll
  for (int r = 0; r < F::VPT / 2; ++r) {
    da[t + r * TL] = v[r].re;
    db[t + r * TL] = v[r].im;
  }
}

// ------------------------------------------------- plane-fused passes ---
// When a z plane's half spectrum fits in LDS (32 <= N <= 128 in FP32,
// N <= 64 in FP64; at N = 128 half a plane, below) the forward x and y
// transforms of one plane run in one block, and so do the inverse y and x
// ones: a solve is three passes (plane forward, z, plane inverse) instead
// of five, and the x-transformed planes never go to memory.  A length-2N
// transform of N nonzero inputs is two length-N transforms,
// F(2m) = DFT_N(f)(m) and F(2m+1) = DFT_N(f w^n)(m) with
// w = exp(-2 pi i / 2N); the first N outputs of a length-2N inverse are
// f(n) = IDFT_N(F(2m))(n) + w^-n IDFT_N(F(2m+1))(n).  So every exchange of
// a line stays within the N slots of LDS the line occupies.
// The plane's spectrum in LDS is column-major, slot(kx, y) = col(kx) +
// pad(y) for kx < N; column 0 holds X(0) + i X(N), both real for a real
// row.  Between the passes the spectra are P[kx][z][ky'] (kx <= N, in the
// C and D buffers), ky' = m for ky = 2m and N + m for ky = 2m + 1: a plane
// writes one 2N run per kx, and a z tile reads within one kx slab.
template <typename T>
struct PadLine {  // one line of LDS in natural order, one pad per 16
  C2<T>* b;
  __device__ __forceinline__ C2<T> ld(int pos) const { return b[pad(pos)]; }
  __device__ __forceinline__ void st(int pos, const C2<T>& x) const { b[pad(pos)] = x; }
};
// Start of column kx in the plane: pitch PC, and 8 more slots for every 16
// columns, so that the lanes of a line that touch positions 16 apart along
// a row (the first Stockham pass) fall in different LDS banks.
__device__ __forceinline__ int pl_col(int kx, int pc) { return kx * pc + (kx >> 4) * 8; }

template <typename T>
struct StrLine {  // one row of the plane: position kx at column kx
  C2<T>* b;
  int s;
  __device__ __forceinline__ C2<T> ld(int pos) const { return b[pl_col(pos, s)]; }
  __device__ __forceinline__ void st(int pos, const C2<T>& x) const { b[pl_col(pos, s)] = x; }
};

template <typename T, int L, int V, int p, class S>
__device__ __forceinline__ void gather_in_g(const S& s, int t, C2<T>* v) {
  constexpr int R = Line<T, L, V>::template R<p>, BPT = Line<T, L, V>::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = s.ld(pos_in<T, L, V, p>(t + b * Line<T, L, V>::TL, r));
}
template <typename T, int L, int V, int p, class S>
__device__ __forceinline__ void scatter_out_g(const S& s, int t, const C2<T>* v) {
  constexpr int R = Line<T, L, V>::template R<p>, BPT = Line<T, L, V>::VPT / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) s.st(pos_out<T, L, V, p>(t + b * Line<T, L, V>::TL, r), v[b * R + r]);
}

// Forward transform of a line (inputs in v at positions t + r TL, natural
// order), the line's LDS slots as exchange space; outputs in v at the last
// pass's natural positions, also stored to the slots when STORE.
template <typename T, int L, int V, int PS, bool STORE, class S>
__device__ __forceinline__ void fwd_from_g(const S& s, int t, C2<T>* v, const C2<T>* __restrict__ tw) {
  constexpr int NP = Line<T, L, V>::NP;
  fwd_bfly<T, L, V, PS>(v, t, tw);
  if constexpr (PS + 1 < NP) {
    scatter_out_g<T, L, V, PS>(s, t, v);
    wave_sync();
    gather_in_g<T, L, V, PS + 1>(s, t, v);
    wave_sync();
    fwd_from_g<T, L, V, PS + 1, STORE>(s, t, v, tw);
  } else if constexpr (STORE) {
    scatter_out_g<T, L, V, PS>(s, t, v);
  }
}

template <typename T, int N>
struct PL {
  static constexpr int V = 16;                     // values per lane of a length-N line
  static constexpr int TL = N / V;                 // lanes per line
  static constexpr int NPL = Line<T, N, V>::NP;
  static constexpr int RL = Line<T, N, V>::template R<NPL - 1>;
  static constexpr int NB = N / RL;                // spacing of the last pass's outputs
  static constexpr int PC = N + N / 16 + 1;        // column pitch
  static constexpr int XP = 2 * N + (2 * N) / 16 + 1;
  static constexpr int XL = N * PC + (N / 16) * 8;  // the plane (skewed columns)
  static constexpr int LDS = XL + XP;              // and column 0's 2N spectrum
  static constexpr bool fits = N >= 32 && N <= 128 && LDS * (int)sizeof(C2<T>) <= 160 * 1024;
};

// Output position of register b * RL + r after a length-N transform.
template <typename T, int N>
__device__ __forceinline__ int pl_pos(int t, int b, int r) {
  return t + b * PL<T, N>::TL + r * PL<T, N>::NB;
}

// Forward: plane z of solve item / N, rho -> P[kx][z][ky'].
template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT)
    k_plane_fwd(const SolveDesc<T>* __restrict__ solves, int* __restrict__ reset,
                const C2<T>* __restrict__ tw, const C2<T>* __restrict__ twist) {
  using G = PL<T, N>;
  constexpr int V = G::V, TL = G::TL, PC = G::PC, RL = G::RL, L = 2 * N;
  constexpr int GROUPS = NT / TL;
  __shared__ C2<T> s[G::LDS];
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;
  const SolveDesc<T>& d = solves[blockIdx.x / N];
  const int z = blockIdx.x % N;
  const int tid = threadIdx.x, t = tid % TL, grp = tid / TL;
  // x: rows 2j and 2j+1 as one complex line; task (j, h) takes the even
  // (h = 0) or odd (h = 1) outputs, with row 2j + h as its exchange space
  // and the place of its outputs.  Below N = 128 the rows of a wavefront's
  // tasks (GPW rows, 1024 values, contiguous) are loaded by the whole
  // wavefront, 16 consecutive values per lane, and staged as
  // z = row 2j + i row 2j+1 in row 2j's slots, where both tasks of the pair
  // take their inputs.  Every round is loaded before the first transform.
  constexpr int GPW = 64 / TL;  // tasks of one wavefront: GPW / 2 row pairs
  constexpr int XR = (N + GROUPS - 1) / GROUPS;
  const int lane = tid & 63, wt0 = (tid >> 6) * GPW;
  if constexpr (N >= 128) {
    // at N = 128 each task loads its own pair of rows (measured faster:
    // the staging's strided LDS writes cost more than the shorter loads save)
    C2<T> xv[XR][V];
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int task = grp + u * GROUPS;
      if (task < N) {
        const size_t row = ((size_t)z * N + 2 * (task >> 1)) * N;
        const gp<const T> a = glb(d.rho + row), b = a + N;
#pragma unroll
        for (int r = 0; r < V; ++r)
          xv[u][r] = C2<T>{__builtin_nontemporal_load(&a[t + r * TL]), __builtin_nontemporal_load(&b[t + r * TL])};
        if (d.rho2) {  // summed grids: the second source is added on the way in
          const gp<const T> a2 = glb(d.rho2 + row), b2 = a2 + N;
#pragma unroll
          for (int r = 0; r < V; ++r) {
            xv[u][r].re += __builtin_nontemporal_load(&a2[t + r * TL]);
            xv[u][r].im += __builtin_nontemporal_load(&b2[t + r * TL]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int task = grp + u * GROUPS;
      if (task < N) {
        const int j = task >> 1, h = task & 1;
        if (h) {
#pragma unroll
          for (int r = 0; r < V; ++r) xv[u][r] = cmul(xv[u][r], twist[t + r * TL]);
        }
        fwd_from_g<T, N, V, 0, true>(StrLine<T>{s + pad(2 * j + h), PC}, t, xv[u], tw);
      }
    }
  } else {
    typedef T t4 __attribute__((ext_vector_type(4)));
    t4 raw[XR][4];
    const int rr = (16 * lane) / N, n0 = (16 * lane) % N;  // row in the wave's block, first column
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int y0 = wt0 + u * GROUPS;  // first row of the wave's block (tasks 2 per row pair)
      if (y0 < N) {
        const gp<const t4> a = (gp<const t4>)glb(d.rho + ((size_t)z * N + y0 + rr) * N + n0);
#pragma unroll
        for (int k = 0; k < 4; ++k) raw[u][k] = __builtin_nontemporal_load(&a[k]);
        if (d.rho2) {  // summed grids: the second source is added on the way in
          const gp<const t4> a2 = (gp<const t4>)glb(d.rho2 + ((size_t)z * N + y0 + rr) * N + n0);
#pragma unroll
          for (int k = 0; k < 4; ++k) raw[u][k] += __builtin_nontemporal_load(&a2[k]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int y0 = wt0 + u * GROUPS;
      const int task = grp + u * GROUPS;
      if (y0 < N) {
        // stage: row y0 + rr holds the real (even row) or imaginary (odd row)
        // part of its pair's line
        const int yr = y0 + rr;
        T* line = (T*)(s + pad(yr & ~1)) + (yr & 1);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int e = 0; e < 4; ++e) line[2 * pl_col(n0 + 4 * k + e, PC)] = raw[u][k][e];
        wave_sync();
        const int j = task >> 1, h = task & 1;
        C2<T> v[V];
#pragma unroll
        for (int r = 0; r < V; ++r) {
          v[r] = s[pl_col(t + r * TL, PC) + pad(2 * j)];
          if (h) v[r] = cmul(v[r], twist[t + r * TL]);
        }
        wave_sync();
        fwd_from_g<T, N, V, 0, true>(StrLine<T>{s + pad(2 * j + h), PC}, t, v, tw);
      }
    }
  }
  __syncthreads();
  // y: column kx (zero-padded to 2N) -> even and odd frequencies; column 0
  // (X(0) + i X(N)) is separated by symmetry through the extra line.
  // A column's values come straight from the two rows' spectra Z of the
  // x transforms (Z = F(row 2j + i row 2j+1)):
  // X_2j(k) = (Z(k) + conj Z(-k)) / 2, X_2j+1(k) = -i (Z(k) - conj Z(-k)) / 2,
  // Z(k) in row 2j (k even) or 2j + 1 (k odd) at k / 2.  Every column reads
  // its values before any column's transform uses its slots.
  // Each half spectrum of a column is staged in the column's own slots and
  // the wavefront writes its columns out whole, 64 lanes in one run, rather
  // than each line's lanes writing their own scattered 64-byte pieces.
  auto zat = [&](int j, int k) -> C2<T> {
    return s[pl_col(k >> 1, PC) + pad(2 * j + (k & 1))];
  };
  const T hf = (T)0.5;
  constexpr int YR = (N + GROUPS - 1) / GROUPS;
  const int wc0 = wt0;  // first column of the wavefront (GPW columns)
  C2<T> uy[YR][V];
#pragma unroll
  for (int yr = 0; yr < YR; ++yr) {
    const int kx = yr * GROUPS + grp;
    if (yr * GROUPS + wc0 < N) {
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int y = t + r * TL, j = y >> 1;
        const C2<T> Z = zat(j, kx), R = zat(j, kx == 0 ? N : L - kx);
        if (kx == 0)  // X(0) and X(N) of the row, real: packed
          uy[yr][r] = (y & 1) ? C2<T>{Z.im, R.im} : C2<T>{Z.re, R.re};
        else
          uy[yr][r] = (y & 1) ? C2<T>{(Z.im + R.im) * hf, (R.re - Z.re) * hf}
                              : C2<T>{(Z.re + R.re) * hf, (Z.im - R.im) * hf};
      }
    }
  }
  __syncthreads();
  C2<T>* const xl = s + G::XL;
#pragma unroll
  for (int yr = 0; yr < YR; ++yr) {
    const int k0 = yr * GROUPS;
    if (k0 + wc0 >= N) break;  // the whole wavefront is past the last column
    const int kx = k0 + grp;
    C2<T>* col = s + pl_col(kx, PC);
    C2<T>* u = uy[yr];
    C2<T> v[V];
#pragma unroll
    for (int r = 0; r < V; ++r) v[r] = u[r];
    wave_sync();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) {
#pragma unroll
        for (int r = 0; r < V; ++r) v[r] = cmul(u[r], twist[t + r * TL]);
        wave_sync();
      }
      fwd_from_g<T, N, V, 0, false>(PadLine<T>{col}, t, v, tw);
      wave_sync();
#pragma unroll
      for (int b = 0; b < V / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int m = pl_pos<T, N>(t, b, r);
          if (kx == 0) xl[pad(h * N + m)] = v[b * RL + r];
          else col[pad(m)] = v[b * RL + r];
        }
      wave_sync();
      for (int c = 0; c < GPW; ++c) {
        const int kc = k0 + wc0 + c;
        if (kc == 0) continue;  // column 0 is separated below
        const C2<T>* cc = s + pl_col(kc, PC);
        const gp<C2<T>> o = glb(d.C + ((size_t)kc * N + z) * L + h * N);
        for (int q = lane; q < N; q += 64) gst(o + q, cc[pad(q)]);
      }
      wave_sync();
    }
    if (kx == 0) {
      wave_sync();
      const gp<C2<T>> o0 = glb(d.C + (size_t)z * L), oN = o0 + (size_t)N * N * L;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < V; ++r) {
          const int m = t + r * TL;
          // mirror -ky (mod 2N) of ky = 2m + h
          const int mm = h ? N - 1 - m : (N - m) & (N - 1);
          const C2<T> A = xl[pad(h * N + m)], B = xl[pad(h * N + mm)];
          gst(o0 + h * N + m, C2<T>{(A.re + B.re) * hf, (A.im - B.im) * hf});
          gst(oN + h * N + m, C2<T>{(A.im + B.im) * hf, (B.re - A.re) * hf});
        }
    }
  }
}

// Forward over half a plane per block.  The columns kx of one parity take
// their row spectra from only one of the two length-N transforms of each
// row pair (the even outputs F(2m) or the odd ones F(2m+1) of the 2N
// line), and the mirror -kx has the same parity; so block parity hp
// transforms every row pair once, for its own outputs, and then the N/2
// columns kx = 2 kx' + hp along y.  The two blocks of a plane share the
// rows' loads only.  A block needs about half the LDS of the whole plane,
// so in FP32 two run on one CU and one's loads and stores overlap the
// other's transforms (in FP64, whose whole plane does not fit, one runs).
// Blocks 8 apart (one XCD) take the two halves of a plane, so the second
// finds the rows in that XCD's L2.
template <typename T, int N>
struct PH {
  static constexpr int V = 16, TL = N / V;
  static constexpr int H = N / 2;                // row pairs; columns per block
  static constexpr int PCX = H + H / 16 + 1;     // x: column m holds the pairs' outputs m
  static constexpr int PC = PL<T, N>::PC;        // y: column kx' holds y = 0..N-1
  static constexpr int XLX = N * PCX + (N / 16) * 8;
  static constexpr int XLY = H * PC + (H / 16) * 8;
  static constexpr int XL = XLX > XLY ? XLX : XLY;
  static constexpr int XP = PL<T, N>::XP;
  static constexpr int LDS = XL + XP;
  // FP32: two blocks per CU; FP64 (whose whole plane does not fit): one
  static constexpr bool fits = N == 128 && LDS * (int)sizeof(C2<T>) * (sizeof(T) == 4 ? 2 : 1) <= 160 * 1024;
};

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT)
    k_plane_fwd_h(const SolveDesc<T>* __restrict__ solves, int* __restrict__ reset,
                  const C2<T>* __restrict__ tw, const C2<T>* __restrict__ twist) {
  using G = PH<T, N>;
  constexpr int V = G::V, TL = G::TL, H = G::H, PCX = G::PCX, PC = G::PC, L = 2 * N;
  constexpr int RL = PL<T, N>::RL, GROUPS = NT / TL, GPW = 64 / TL;
  static_assert(H % GPW == 0 && GROUPS % GPW == 0, "a wavefront's columns lie in one round");
  __shared__ C2<T> s[G::LDS];
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;
  const int bq = blockIdx.x >> 3, hp = bq & 1;
  const int plane = (bq >> 1) * 8 + (blockIdx.x & 7);
  const SolveDesc<T>& d = solves[plane / N];
  const int z = plane % N;
  const int tid = threadIdx.x, t = tid % TL, grp = tid / TL, lane = tid & 63;
  const int wc0 = (tid >> 6) * GPW;  // first column of the wavefront in a round
  // x: task j, rows 2j + i row 2j+1 (times w^n for the odd outputs); its
  // outputs m go to position j of column m
  constexpr int XR = (H + GROUPS - 1) / GROUPS;
  C2<T> xv[XR][V];
#pragma unroll
  for (int u = 0; u < XR; ++u) {
    const int j = grp + u * GROUPS;
    if (j < H) {
      const size_t row = ((size_t)z * N + 2 * j) * N;
      const gp<const T> a = glb(d.rho + row), b = a + N;
#pragma unroll
      for (int r = 0; r < V; ++r) xv[u][r] = C2<T>{a[t + r * TL], b[t + r * TL]};
      if (d.rho2) {  // summed grids: the second source is added on the way in
        const gp<const T> a2 = glb(d.rho2 + row), b2 = a2 + N;
#pragma unroll
        for (int r = 0; r < V; ++r) {
          xv[u][r].re += a2[t + r * TL];
          xv[u][r].im += b2[t + r * TL];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < XR; ++u) {
    const int j = grp + u * GROUPS;
    if (j < H) {
      if (hp) {
#pragma unroll
        for (int r = 0; r < V; ++r) xv[u][r] = cmul(xv[u][r], twist[t + r * TL]);
      }
      fwd_from_g<T, N, V, 0, true>(StrLine<T>{s + pad(j), PCX}, t, xv[u], tw);
    }
  }
  __syncthreads();
  // y: as in the whole-plane form, Z(k) of pair j is at position j of
  // column k / 2 (k of parity hp, as is its mirror 2N - k)
  auto zat = [&](int j, int k) -> C2<T> { return s[pl_col(k >> 1, PCX) + pad(j)]; };
  const T hf = (T)0.5;
  constexpr int YR = (H + GROUPS - 1) / GROUPS;
  C2<T> uy[YR][V];
#pragma unroll
  for (int yr = 0; yr < YR; ++yr) {
    const int kx = 2 * (yr * GROUPS + grp) + hp;
    if (yr * GROUPS + wc0 < H) {
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int y = t + r * TL, j = y >> 1;
        const C2<T> Z = zat(j, kx), R = zat(j, kx == 0 ? N : L - kx);
        if (kx == 0)  // X(0) and X(N) of the row, real: packed
          uy[yr][r] = (y & 1) ? C2<T>{Z.im, R.im} : C2<T>{Z.re, R.re};
        else
          uy[yr][r] = (y & 1) ? C2<T>{(Z.im + R.im) * hf, (R.re - Z.re) * hf}
                              : C2<T>{(Z.re + R.re) * hf, (Z.im - R.im) * hf};
      }
    }
  }
  __syncthreads();
  C2<T>* const xl = s + G::XL;
#pragma unroll
  for (int yr = 0; yr < YR; ++yr) {
    const int k0 = yr * GROUPS;
    if (k0 + wc0 >= H) break;  // the whole wavefront is past the last column
    const int kq = k0 + grp, kx = 2 * kq + hp;
    C2<T>* col = s + pl_col(kq, PC);
    C2<T>* u = uy[yr];
    C2<T> v[V];
#pragma unroll
    for (int r = 0; r < V; ++r) v[r] = u[r];
    wave_sync();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) {
#pragma unroll
        for (int r = 0; r < V; ++r) v[r] = cmul(u[r], twist[t + r * TL]);
        wave_sync();
      }
      fwd_from_g<T, N, V, 0, false>(PadLine<T>{col}, t, v, tw);
      wave_sync();
#pragma unroll
      for (int b = 0; b < V / RL; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int m = pl_pos<T, N>(t, b, r);
          if (kx == 0) xl[pad(h * N + m)] = v[b * RL + r];
          else col[pad(m)] = v[b * RL + r];
        }
      wave_sync();
      for (int c = 0; c < GPW; ++c) {
        const int cq = k0 + wc0 + c, kc = 2 * cq + hp;
        if (kc == 0) continue;  // column 0 is separated below
        const C2<T>* cc = s + pl_col(cq, PC);
        const gp<C2<T>> o = glb(d.C + ((size_t)kc * N + z) * L + h * N);
        for (int q = lane; q < N; q += 64) gst(o + q, cc[pad(q)]);
      }
      wave_sync();
    }
    if (kx == 0) {
      wave_sync();
      const gp<C2<T>> o0 = glb(d.C + (size_t)z * L), oN = o0 + (size_t)N * N * L;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < V; ++r) {
          const int m = t + r * TL;
          const int mm = h ? N - 1 - m : (N - m) & (N - 1);
          const C2<T> A = xl[pad(h * N + m)], B = xl[pad(h * N + mm)];
          gst(o0 + h * N + m, C2<T>{(A.re + B.re) * hf, (A.im - B.im) * hf});
          gst(oN + h * N + m, C2<T>{(A.im + B.im) * hf, (B.re - A.re) * hf});
        }
    }
  }
}

// Inverse: P[kx][z][ky'] (the z pass's output, D) -> phi plane z (x, y < N).
template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT)
    k_plane_inv(const SolveDesc<T>* __restrict__ solves, int* __restrict__ reset,
                const C2<T>* __restrict__ tw, const C2<T>* __restrict__ twist) {
  using G = PL<T, N>;
  constexpr int V = G::V, TL = G::TL, PC = G::PC, RL = G::RL, L = 2 * N;
  constexpr int GROUPS = NT / TL;
  __shared__ C2<T> s[G::LDS];
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;
  const SolveDesc<T>& d = solves[blockIdx.x / N];
  const int z = blockIdx.x % N;
  const int tid = threadIdx.x, t = tid % TL, grp = tid / TL;
  // y: column kx from its even and odd frequencies (column 0 from
  // Q(0) + i Q(N), whose inverse is X(0) + i X(N)); inverse transforms as
  // conj(F(conj .)), unnormalised
  // The wavefront loads its columns' inputs whole, 64 lanes in one run
  // (both halves before the first transform), and stages each half in the
  // columns' slots, from where each line takes its own values.
  constexpr int GPW = 64 / TL;
  constexpr int QPL = (N + 63) / 64;  // values per lane of one column half
  const int lane = tid & 63, wc0 = (tid >> 6) * GPW;
#pragma unroll 1
  for (int k0 = 0; k0 < N; k0 += GROUPS) {
    if (k0 + wc0 >= N) break;  // the whole wavefront is past the last column
    const int kx = k0 + grp;
    C2<T>* col = s + pl_col(kx, PC);
    C2<T> pre[2][GPW][QPL];
#pragma unroll
    for (int c = 0; c < GPW; ++c) {
      const int kc = k0 + wc0 + c;
      const gp<const C2<T>> q = glb(d.D + ((size_t)kc * N + z) * L);
      const gp<const C2<T>> qn = glb(d.D + ((size_t)N * N + z) * L);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < QPL; ++k) {
          const int m = lane + 64 * k;
          if (m < N) {
            C2<T> e{__builtin_nontemporal_load(&q[h * N + m].re), __builtin_nontemporal_load(&q[h * N + m].im)};
            if (kc == 0) {  // Q(0) + i Q(N)
              const C2<T> f{__builtin_nontemporal_load(&qn[h * N + m].re),
                            __builtin_nontemporal_load(&qn[h * N + m].im)};
              e = C2<T>{e.re - f.im, e.im + f.re};
            }
            pre[h][c][k] = e;
          }
        }
    }
    C2<T> a[V], v[V];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) wave_sync();
#pragma unroll
      for (int c = 0; c < GPW; ++c)
#pragma unroll
        for (int k = 0; k < QPL; ++k)
          if (lane + 64 * k < N) s[pl_col(k0 + wc0 + c, PC) + pad(lane + 64 * k)] = pre[h][c][k];
      wave_sync();
#pragma unroll
      for (int r = 0; r < V; ++r) v[r] = conjc(col[pad(t + r * TL)]);
      wave_sync();
      fwd_from_g<T, N, V, 0, false>(PadLine<T>{col}, t, v, tw);
      if (!h) {
#pragma unroll
        for (int i = 0; i < V; ++i) a[i] = conjc(v[i]);
      }
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < V / RL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int y = pl_pos<T, N>(t, b, r), i = b * RL + r;
        col[pad(y)] = a[i] + cmul(conjc(twist[y]), conjc(v[i]));
      }
  }
  __syncthreads();
  // x: rows 2j, 2j+1 as Z = X_a + i X_b, extended to 2N by Hermitian
  // symmetry; task (j, h) gathers Z(2m + h) and transforms it, rows 2j + h
  // as exchange space and output place
  auto xat = [&](int y, int k) -> C2<T> {  // X(k) of row y, 0 <= k <= N
    const C2<T> c = s[pl_col(k == N ? 0 : k, PC) + pad(y)];
    return k == 0 ? C2<T>{c.re, (T)0} : (k == N ? C2<T>{c.im, (T)0} : c);
  };
  constexpr int XR = (N + GROUPS - 1) / GROUPS;
  C2<T> v[XR][V];
#pragma unroll
  for (int u = 0; u < XR; ++u) {
    const int task = grp + u * GROUPS;
    if (task < N) {
      const int j = task >> 1, h = task & 1;
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int k = 2 * (t + r * TL) + h;
        C2<T> zz;
        if (k <= N) {
          const C2<T> A = xat(2 * j, k), B = xat(2 * j + 1, k);
          zz = C2<T>{A.re - B.im, A.im + B.re};
        } else {
          const C2<T> A = xat(2 * j, L - k), B = xat(2 * j + 1, L - k);
          zz = C2<T>{A.re + B.im, B.re - A.im};
        }
        v[u][r] = conjc(zz);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < XR; ++u) {
    const int task = grp + u * GROUPS;
    if (task < N) {
      const int j = task >> 1, h = task & 1;
      fwd_from_g<T, N, V, 0, true>(StrLine<T>{s + pad(2 * j + h), PC}, t, v[u], tw);
    }
  }
  __syncthreads();
  // z(n) = IDFT(even)(n) + w^-n IDFT(odd)(n): real part row 2j, imaginary
  // part row 2j + 1
  const gp<T> ph = glb(d.phi + (size_t)z * N * N);
  for (int i = tid; i < N * N / 2; i += NT) {
    const int j = i / N, n = i - j * N;
    const C2<T> A = conjc(s[pl_col(n, PC) + pad(2 * j)]), B = conjc(s[pl_col(n, PC) + pad(2 * j + 1)]);
    const C2<T> zz = A + cmul(conjc(twist[n]), B);
    ph[(size_t)(2 * j) * N + n] = zz.re;
    ph[(size_t)(2 * j + 1) * N + n] = zz.im;
  }
}

// Inverse over half a plane per block: block parity hp makes the rows
// y = 2p + hp.  Those outputs of a column's length-2N inverse along y come
// from two length-N/2 inverses.  With E and O the column's even and odd ky
// halves and s = (-1)^hp, row 2p + hp is a(p) + w^-(2p+hp) b(p), where
// a = IDFT_{N/2}((E(m) + s E(m + N/2)) e^{2 pi i m hp / N}) and b is the
// same of O.  So a block does half the plane's y transforms (no transform
// is done by both blocks), its N/2 rows pair up for the x phase as in the
// whole-plane form, and only the D columns are read by both blocks of a
// plane (8 apart, on one XCD, so the second mostly reads them from L2).
// The y lines (N/2) use the table twh; the x lines (N) use tw.
template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT)
    k_plane_inv_h(const SolveDesc<T>* __restrict__ solves, int* __restrict__ reset,
                  const C2<T>* __restrict__ tw, const C2<T>* __restrict__ twist,
                  const C2<T>* __restrict__ twh) {
  using G = PH<T, N>;
  constexpr int V = G::V, TL = G::TL, H = G::H, PCX = G::PCX, L = 2 * N;
  static_assert(H == 64, "one lane per value of a y line half");
  constexpr int TLH = H / V, GH = NT / TLH, GPWH = 64 / TLH, RLH = PL<T, H>::RL;
  constexpr int GROUPS = NT / TL;
  __shared__ C2<T> s[G::XLX];
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;
  const int bq = blockIdx.x >> 3, hp = bq & 1;
  const int plane = (bq >> 1) * 8 + (blockIdx.x & 7);
  const SolveDesc<T>& d = solves[plane / N];
  const int z = plane % N;
  const int tid = threadIdx.x, lane = tid & 63;
  // y: column kx at slots col(kx) + pad(p), p = 0..N/2-1.  The wavefront
  // loads its columns whole (lane m takes m and m + N/2 of both halves,
  // column 0 as Q(0) + i Q(N)), folds them, and stages each folded half in
  // the column's slots, from where each line takes its own values.
  {
    const int th = tid % TLH, gh = tid / TLH, wc0 = (tid >> 6) * GPWH;
    const T sg = hp ? (T)-1 : (T)1;
    const C2<T> tm = hp ? conjc(twist[2 * lane]) : C2<T>{(T)1, (T)0};
#pragma unroll 1
    for (int k0 = 0; k0 < N; k0 += GH) {
      if (k0 + wc0 >= N) break;  // the whole wavefront is past the last column
      const int kx = k0 + gh;
      C2<T>* col = s + pl_col(kx, PCX);
      C2<T> pre[2][GPWH];
#pragma unroll
      for (int c = 0; c < GPWH; ++c) {
        const int kc = k0 + wc0 + c;
        const gp<const C2<T>> q = glb(d.D + ((size_t)kc * N + z) * L);
        const gp<const C2<T>> qn = glb(d.D + ((size_t)N * N + z) * L);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          C2<T> e0 = gld(q + (h * N + lane)), e1 = gld(q + (h * N + H + lane));
          if (kc == 0) {  // Q(0) + i Q(N)
            const C2<T> f0 = gld(qn + (h * N + lane)), f1 = gld(qn + (h * N + H + lane));
            e0 = C2<T>{e0.re - f0.im, e0.im + f0.re};
            e1 = C2<T>{e1.re - f1.im, e1.im + f1.re};
          }
          const C2<T> x{e0.re + sg * e1.re, e0.im + sg * e1.im};
          pre[h][c] = hp ? cmul(x, tm) : x;
        }
      }
      C2<T> a[V], v[V];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h) wave_sync();
#pragma unroll
        for (int c = 0; c < GPWH; ++c) s[pl_col(k0 + wc0 + c, PCX) + pad(lane)] = pre[h][c];
        wave_sync();
#pragma unroll
        for (int r = 0; r < V; ++r) v[r] = conjc(col[pad(th + r * TLH)]);
        wave_sync();
        fwd_from_g<T, H, V, 0, false>(PadLine<T>{col}, th, v, twh);
        if (!h) {
#pragma unroll
          for (int i = 0; i < V; ++i) a[i] = conjc(v[i]);
        }
      }
      wave_sync();
#pragma unroll
      for (int b = 0; b < V / RLH; ++b)
#pragma unroll
        for (int r = 0; r < RLH; ++r) {
          const int pp = pl_pos<T, H>(th, b, r), i = b * RLH + r;
          col[pad(pp)] = a[i] + cmul(conjc(twist[2 * pp + hp]), conjc(v[i]));
        }
    }
  }
  __syncthreads();
  // x: the block's rows 2j and 2j+1 (y = 4j + hp and 4j + 2 + hp) as
  // Z = X_a + i X_b, as in the whole-plane form; task 2j + h its exchange
  // space and output place
  const int t = tid % TL, grp = tid / TL;
  auto xat = [&](int p, int k) -> C2<T> {  // X(k) of block row p, 0 <= k <= N
    const C2<T> c = s[pl_col(k == N ? 0 : k, PCX) + pad(p)];
    return k == 0 ? C2<T>{c.re, (T)0} : (k == N ? C2<T>{c.im, (T)0} : c);
  };
  constexpr int XR = (H + GROUPS - 1) / GROUPS;
  C2<T> v[XR][V];
#pragma unroll
  for (int u = 0; u < XR; ++u) {
    const int task = grp + u * GROUPS;
    if (task < H) {
      const int j = task >> 1, h = task & 1;
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int k = 2 * (t + r * TL) + h;
        C2<T> zz;
        if (k <= N) {
          const C2<T> A = xat(2 * j, k), B = xat(2 * j + 1, k);
          zz = C2<T>{A.re - B.im, A.im + B.re};
        } else {
          const C2<T> A = xat(2 * j, L - k), B = xat(2 * j + 1, L - k);
          zz = C2<T>{A.re + B.im, B.re - A.im};
        }
        v[u][r] = conjc(zz);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < XR; ++u) {
    const int task = grp + u * GROUPS;
    if (task < H) fwd_from_g<T, N, V, 0, true>(StrLine<T>{s + pad(task), PCX}, t, v[u], tw);
  }
  __syncthreads();
  const gp<T> ph = glb(d.phi + (size_t)z * N * N);
  for (int i = tid; i < (H / 2) * N; i += NT) {
    const int j = i / N, n = i - j * N;
    const C2<T> A = conjc(s[pl_col(n, PCX) + pad(2 * j)]), B = conjc(s[pl_col(n, PCX) + pad(2 * j + 1)]);
    const C2<T> zz = A + cmul(conjc(twist[n]), B);
    ph[(size_t)(4 * j + hp) * N + n] = zz.re;
    ph[(size_t)(4 * j + 2 + hp) * N + n] = zz.im;
  }
}

template <typename T, int L, int V, int NT, int PASS>
__device__ __forceinline__ void run_tile(const SolveDesc<T>& d, int tile, C2<T>* s,
                                         const C2<T>* __restrict__ tw) {
  if constexpr (PASS == 0) tile_fwd_x<T, L, V, NT>(d, tile, s, tw);
  else if constexpr (PASS == 1) tile_fwd_y<T, L, V, NT>(d, tile, s, tw);
  else if constexpr (PASS == 2) tile_zpass<T, L, V, NT, false>(d, tile, s, tw);
  else if constexpr (PASS == 5) tile_zpass<T, L, V, NT, true>(d, tile, s, tw);
  else if constexpr (PASS == 3) tile_inv_y<T, L, V, NT>(d, tile, s, tw);
  else tile_inv_x<T, L, V, NT>(d, tile, s, tw);
}

// Persistent pass over the solves of one grid size: work items are
// (solve, tile) pairs; the first item of a block is its index, later ones
// come from the counter until all are done.  With one block per item the
// counter is never touched.  `reset` (may be null) is the counter of the
// pass that ran before this one; it is cleared here for its next use, which
// saves a launch per solve set.
template <typename T, int PASS, int NT, int L, int V>
__global__ void __launch_bounds__(NT)
    k_pass(const SolveDesc<T>* __restrict__ solves, int tiles_per_solve, int total,
           int* __restrict__ counter, int* __restrict__ reset, const C2<T>* __restrict__ tw) {
  __shared__ C2<T> s[TC<T, L, V, NT, PASS>::LDS];
  __shared__ int item_sh;
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;
  int next = blockIdx.x;
  for (;;) {
    const int item = next;
    if (item >= total) break;
    const bool more = (int)gridDim.x < total;
    if (more && threadIdx.x == 0) item_sh = (int)gridDim.x + atomicAdd(counter, 1);
    const int sidx = item / tiles_per_solve;
    run_tile<T, L, V, NT, PASS>(solves[sidx], item - sidx * tiles_per_solve, s, tw);
    if (!more) break;
    __syncthreads();  // LDS free for the next tile; item_sh written
    next = __builtin_amdgcn_readfirstlane(item_sh);
    __syncthreads();  // item_sh read by all before thread 0 rewrites it
  }
}

// Calls f(L, V) (as integral constants) for the line length of N^3 grids
// and the schedule v (0 or a value the line length does not have: its
// default schedule).
template <typename T, typename Fn>
static auto with_lv(int N, int v, Fn&& f) {
  auto pick = [&](auto lc) {
    constexpr int L = decltype(lc)::value;
    if constexpr (kTwoV<T, L>) {
      if (v == 16) return f(lc, std::integral_constant<int, 16>());
      if (v == 32) return f(lc, std::integral_constant<int, 32>());
    }
    return f(lc, std::integral_constant<int, kDefV<T, L>>());
  };
  switch (N) {
    case 8: return pick(std::integral_constant<int, 16>());
    case 16: return pick(std::integral_constant<int, 32>());
    case 32: return pick(std::integral_constant<int, 64>());
    case 64: return pick(std::integral_constant<int, 128>());
    case 128: return pick(std::integral_constant<int, 256>());
    default: return pick(std::integral_constant<int, 512>());
  }
}

// The same for the block size (128, 256 or 512).
template <typename Fn>
static auto with_nt(int nt, Fn&& f) {
  if (nt == 128) return f(std::integral_constant<int, 128>());
  if (nt == 256) return f(std::integral_constant<int, 256>());
  return f(std::integral_constant<int, 512>());
}

template <typename T>
static int tiles_nt(int nt, int v, int N, int pass) {
  return with_nt(nt, [&](auto ntc) {
    return with_lv<T>(N, v, [&](auto lc, auto vc) {
      return tiles_of<T, decltype(lc)::value, decltype(vc)::value, decltype(ntc)::value>(pass);
    });
  });
}

// Whether a block size and schedule fit the LDS budget for a pass and grid
// size.
template <typename T>
static bool shape_ok(int nt, int v, int N, int pass) {
  if (nt != 128 && nt != 256 && nt != 512) return false;
  return with_nt(nt, [&](auto ntc) {
    return with_lv<T>(N, v, [&](auto lc, auto vc) {
      constexpr int L = decltype(lc)::value, V = decltype(vc)::value, NT = decltype(ntc)::value;
      switch (pass) {
        case 0: return shape_fits<T, L, V, NT, 0>();
        case 1: return shape_fits<T, L, V, NT, 1>();
        case 2:
        case 5: return shape_fits<T, L, V, NT, 2>();
        case 3: return shape_fits<T, L, V, NT, 3>();
        default: return shape_fits<T, L, V, NT, 4>();
      }
    });
  });
}

template <typename T, int PASS>
static void launch_pass(const SolveDesc<T>* solves, int N, int nsolves, PassShape sh, int* counter,
                        int* reset, const C2<T>* tw, hipStream_t st) {
  if (!shape_ok<T>(sh.nt, sh.v, N, PASS)) sh = PassShape{256, sh.grid, 0};
  const int tps = tiles_nt<T>(sh.nt, sh.v, N, PASS);
  const int total = tps * nsolves;
  const int grid = std::max(1, std::min(sh.grid <= 0 ? total : sh.grid, total));
  with_nt(sh.nt, [&](auto ntc) {
    with_lv<T>(N, sh.v, [&](auto lc, auto vc) {
      constexpr int L = decltype(lc)::value, V = decltype(vc)::value, NT = decltype(ntc)::value;
      hipLaunchKernelGGL((k_pass<T, PASS, NT, L, V>), dim3(grid), dim3(NT), 0, st, solves, tps, total,
                         counter, reset, tw);
    });
  });
}

template <typename T>
static void launch_any(int pass, const SolveDesc<T>* solves, int N, int nsolves, PassShape sh,
                       int* counter, int* reset, const C2<T>* tw, hipStream_t st) {
  switch (pass) {
    case 0: launch_pass<T, 0>(solves, N, nsolves, sh, counter, reset, tw, st); break;
    case 1: launch_pass<T, 1>(solves, N, nsolves, sh, counter, reset, tw, st); break;
    case 2: launch_pass<T, 2>(solves, N, nsolves, sh, counter, reset, tw, st); break;
    case 3: launch_pass<T, 3>(solves, N, nsolves, sh, counter, reset, tw, st); break;
    case 5: launch_pass<T, 5>(solves, N, nsolves, sh, counter, reset, tw, st); break;
    default: launch_pass<T, 4>(solves, N, nsolves, sh, counter, reset, tw, st); break;
  }
}

__global__ void k_zero_int(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// w^n = exp(-2 pi i n / 2N), n < N: the twist between the even and odd
// halves of a zero-padded length-2N transform (FP64, then rounded).
template <typename T>
__global__ void k_twist(C2<T>* w, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double sn, cs;
  sincospi((double)n / (double)N, &sn, &cs);
  w[n] = C2<T>{(T)cs, (T)(-sn)};
}

// Twist tables, like the twiddle tables made once per (device, precision,
// N) and kept; with create = false a missing one is not made.
template <typename T>
static const C2<T>* twist_table(int N, hipStream_t st, bool create = true) {
  static std::mutex mu;
  static C2<T>* cache[64][10] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  int lg = 0;
  while ((1 << lg) < N) ++lg;
  std::lock_guard<std::mutex> g(mu);
  if (cache[dev][lg] || !create) return cache[dev][lg];
  C2<T>* p = nullptr;
  if (hipMalloc(&p, sizeof(C2<T>) * N) != hipSuccess) return nullptr;
  hipLaunchKernelGGL(k_twist<T>, dim3((N + 255) / 256), dim3(256), 0, st, p, N);
  if (hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(p);
    return nullptr;
  }
  cache[dev][lg] = p;
  return p;
}

// Whether the plane-fused form exists for this precision and size, and
// for this block size.
template <typename T>
static bool plane_ok(int N) {
  return (N == 32 && PL<T, 32>::fits) || (N == 64 && PL<T, 64>::fits) ||
         (N == 128 && (PL<T, 128>::fits || PH<T, 128>::fits));
}
template <typename T>
static bool plane_nt_ok(int N, int nt, bool inv) {
  // FP64 at 1024 threads would leave too few registers per lane; the
  // half-plane passes have 256 or 512 (the inverse at 1024: whole planes)
  if (!inv && N == 128 && PH<T, 128>::fits) return nt == 256 || nt == 512;
  return plane_ok<T>(N) && (nt == 256 || nt == 512 || (nt == 1024 && sizeof(T) == 4));
}

// Tables of the plane passes: lines of N (16 values per lane), the twist,
// and where the half-plane passes run, the lines of N/2 of the inverse.
template <typename T>
static bool plane_tables(int N, hipStream_t st) {
  if (!twiddles<T>(N, 16, st) || !twist_table<T>(N, st)) return false;
  return !(N == 128 && PH<T, 128>::fits) || twiddles<T>(N / 2, 16, st);
}

template <typename T, int N>
static void launch_plane_n(bool inv, const SolveDesc<T>* solves, int nsolves, int nt, int* reset,
                           const C2<T>* tw, const C2<T>* twist, hipStream_t st) {
  if constexpr (PL<T, N>::fits || PH<T, N>::fits) {
    if constexpr (PH<T, N>::fits) {
      const dim3 grid(2 * nsolves * N);  // half a plane per block
      if (!inv) {  // 256 or 512 threads: 1024 would idle half the groups
        if (nt == 256)
          hipLaunchKernelGGL((k_plane_fwd_h<T, N, 256>), grid, dim3(256), 0, st, solves, reset, tw, twist);
        else
          hipLaunchKernelGGL((k_plane_fwd_h<T, N, 512>), grid, dim3(512), 0, st, solves, reset, tw, twist);
        return;
      }
      // the inverse: 256 or 512 threads take half a plane (its y lines of
      // N/2 need their own table, made with the plan; without it the
      // whole-plane inverse runs), 1024 the whole plane
      const C2<T>* twh = nt == 1024 ? nullptr : twiddles<T>(N / 2, 16, st, false);
      if (twh) {
        if (nt == 256)
          hipLaunchKernelGGL((k_plane_inv_h<T, N, 256>), grid, dim3(256), 0, st, solves, reset, tw, twist, twh);
        else
          hipLaunchKernelGGL((k_plane_inv_h<T, N, 512>), grid, dim3(512), 0, st, solves, reset, tw, twist, twh);
        return;
      }
    }
    if constexpr (PL<T, N>::fits) {  // whole planes (FP64 at N = 128 has none)
      auto go = [&](auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        if (inv)
          hipLaunchKernelGGL((k_plane_inv<T, N, NT>), dim3(nsolves * N), dim3(NT), 0, st, solves, reset, tw,
                             twist);
        else
          hipLaunchKernelGGL((k_plane_fwd<T, N, NT>), dim3(nsolves * N), dim3(NT), 0, st, solves, reset, tw,
                             twist);
      };
      if (nt == 256) go(std::integral_constant<int, 256>());
      else if constexpr (sizeof(T) == 8) go(std::integral_constant<int, 512>());
      else if (nt == 512) go(std::integral_constant<int, 512>());
      else go(std::integral_constant<int, 1024>());
    }
  }
}

template <typename T>
static void launch_plane(bool inv, const SolveDesc<T>* solves, int N, int nsolves, int nt, int* reset,
                         const C2<T>* tw, const C2<T>* twist, hipStream_t st) {
  switch (N) {
    case 32: launch_plane_n<T, 32>(inv, solves, nsolves, nt, reset, tw, twist, st); break;
    case 64: launch_plane_n<T, 64>(inv, solves, nsolves, nt, reset, tw, twist, st); break;
    default: launch_plane_n<T, 128>(inv, solves, nsolves, nt, reset, tw, twist, st); break;
  }
}

// ---------------------------------------------------------- the autotuner --
// Candidate shapes per (precision, grid size, solve count, pass): the line
// schedule (in FP32 for lines of 128 and more: 16 or 32 values per thread,
// that is radix 16 then L/16 (then 2), or radix 32 then L/32), block size
// 128, 256 or 512 threads (where the tile fits the LDS budget) and a
// persistent grid of 2, 4 or 8 blocks per compute unit, or one block per
// tile.  Each candidate runs the pass on the plan's own buffers (zeroed
// first); the fastest of 5 timed repetitions wins.  Results are cached for
// the life of the process.
struct TuneKey {
  int esz, N, count;
  int pin = 0;   // the pinned line schedule when the key was tuned (0: none)
  int fpin = 0;  // the pinned form (3 or 5 passes; 0: none)
  int npin = 0;  // the pinned block size of the plane passes (0: none)
  bool operator==(const TuneKey& o) const {
    return esz == o.esz && N == o.N && count == o.count && pin == o.pin && fpin == o.fpin && npin == o.npin;
  }
};

// What the tuner chose: the form (5: the five line passes; 3: plane
// forward, z pass on the plane layout, plane inverse, whose shapes are
// sh[0], sh[2] and sh[3]) and the launch shape of each pass.
struct Tuned {
  std::array<PassShape, kPasses> sh;
  int form = 5;
  float ms5 = 0.f, ms3 = 0.f;  // the tuner's time of a whole solve set in each form (0: not timed)
};

// Line schedule pinned for plans tuned from now on (0: the tuner times
// every schedule a line length has).
static std::atomic<int> g_pin_v{0};
// Form pinned for plans tuned from now on (0: the tuner times both where
// the plane form exists).
static std::atomic<int> g_pin_form{0};
// Block size of the plane passes pinned for plans tuned from now on (0: the
// tuner times every one a pass has; a pass without the pinned one still
// times its own).
static std::atomic<int> g_pin_nt{0};

sbx_status set_plane_threads(int nt) {
  if (nt != 0 && nt != 256 && nt != 512 && nt != 1024) {
    set_error("plane block size must be 0 (tuned), 256, 512 or 1024");
    return SBX_EINVAL;
  }
  g_pin_nt.store(nt);
  return SBX_OK;
}

sbx_status set_fft_form(int f) {
  if (f != 0 && f != 3 && f != 5) {
    set_error("FFT form must be 0 (tuned), 3 (plane-fused passes) or 5 (five line passes)");
    return SBX_EINVAL;
  }
  g_pin_form.store(f);
  return SBX_OK;
}

sbx_status set_fft_schedule(int v) {
  if (v != 0 && v != 16 && v != 32) {
    set_error("values per thread must be 0 (tuned), 16 or 32");
    return SBX_EINVAL;
  }
  g_pin_v.store(v);
  return SBX_OK;
}

static std::mutex g_tune_mu;
static std::vector<std::pair<TuneKey, Tuned>> g_tune;

static TuneKey key_now(int esz, int N, int count) {
  return TuneKey{esz, N, count, g_pin_v.load(), g_pin_form.load(), g_pin_nt.load()};
}

static bool tune_lookup(const TuneKey& k, Tuned& out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (auto& e : g_tune)
    if (e.first == k) {
      out = e.second;
      return true;
    }
  return false;
}

std::string tuning_report() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::string out;
  static const char* names[kPasses] = {"fwd_x", "fwd_y", "zpass", "inv_y", "inv_x"};
  static const char* pnames[kPasses] = {"plane_fwd", "", "zpass", "plane_inv", ""};
  for (auto& e : g_tune) {
    const bool pl = e.second.form == 3;
    for (int p = 0; p < kPasses; ++p) {
      if (pl && (p == 1 || p == 4)) continue;
      const PassShape& sh = e.second.sh[p];
      out += std::string(e.first.esz == 8 ? "fp64" : "fp32") + " N=" + std::to_string(e.first.N) + " x" +
             std::to_string(e.first.count) + " form=" + std::to_string(e.second.form) + " " +
             (pl ? pnames[p] : names[p]) + " nt=" + std::to_string(sh.nt);
      if (!pl || p == 2)
        out += " grid=" + (sh.grid <= 0 ? std::string("tiles") : std::to_string(sh.grid)) + " v=" +
               std::to_string(e.first.esz == 8 ? eff_v<double>(2 * e.first.N, sh.v)
                                               : eff_v<float>(2 * e.first.N, sh.v));
      out += "\n";
    }
    if (e.second.ms5 > 0.f && e.second.ms3 > 0.f)
      out += std::string(e.first.esz == 8 ? "fp64" : "fp32") + " N=" + std::to_string(e.first.N) + " x" +
             std::to_string(e.first.count) + " form=" + std::to_string(e.second.form) +
             " timed five-pass " + std::to_string(e.second.ms5) + " ms, plane " + std::to_string(e.second.ms3) +
             " ms\n";
  }
  return out;
}

static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
  return cus > 0 ? cus : 256;
}

bool tuning_cached(int esz, std::vector<int> mix) {
  std::sort(mix.begin(), mix.end());
  for (size_t i = 0; i < mix.size();) {
    size_t j = i;
    while (j < mix.size() && mix[j] == mix[i]) ++j;
    Tuned a;
    if (!tune_lookup(key_now(esz, mix[i], (int)(j - i)), a)) return false;
    i = j;
  }
  return true;
}

// One pass of a group in either form.  Plane form: pass 0 is the plane
// forward, 2 the z pass on the plane layout, 3 the plane inverse; 1 and 4
// launch nothing.  Each launch clears the work counter of the pass before.
template <typename T>
static void run_pass(int form, int q, const SolveDesc<T>* solves, int N, int count, const PassShape& sh,
                     int* ctr, int* prev, const C2<T>* tw, const C2<T>* twist, hipStream_t st) {
  if (form != 3) {
    launch_any<T>(q, solves, N, count, sh, ctr, prev, tw, st);
  } else if (q == 0 || q == 3) {
    launch_plane<T>(q == 3, solves, N, count, sh.nt, prev, tw, twist, st);
  } else if (q == 2) {
    launch_any<T>(5, solves, N, count, sh, ctr, prev, tw, st);
  }
}

template <typename T>
static sbx_status tune_group(const SolveDesc<T>* d_solves, const SolveDesc<T>* host, int N, int count,
                             int* counter, hipStream_t st, Tuned& out) {
  const int cus = device_cus();
  const int nts[3] = {128, 256, 512};
  const int bpcs[4] = {2, 4, 8, 0};  // 0: one block per tile
  const int fpin = g_pin_form.load();
  const bool plane = plane_ok<T>(N) && fpin != 5;
  const bool five = !plane || fpin != 3;
  // the schedules of this line length (one, or both 16 and 32)
  const int L = 2 * N;
  std::vector<int> vs{eff_v<T>(L, 0)};
  if (eff_v<T>(L, 16) != eff_v<T>(L, 32)) {
    const int pin = g_pin_v.load();
    vs = pin ? std::vector<int>{pin} : std::vector<int>{16, 32};
  }
  const C2<T>* tws[2] = {nullptr, nullptr};
  for (size_t i = 0; i < vs.size(); ++i) {
    tws[i] = twiddles<T>(L, vs[i], st);
    if (!tws[i]) {
      set_error("twiddle table allocation failed");
      return SBX_ENOMEM;
    }
  }
  const C2<T>* twh = plane ? twiddles<T>(N, 16, st) : nullptr;
  const C2<T>* twist = plane ? twist_table<T>(N, st) : nullptr;
  if (plane && (!twh || !twist || !plane_tables<T>(N, st))) {
    set_error("twiddle table allocation failed");
    return SBX_ENOMEM;
  }
  for (int i = 0; i < count; ++i) {
    SBX_HIP(hipMemsetAsync((void*)host[i].rho, 0, sizeof(T) * (size_t)N * N * N, st));
    if (host[i].rho2)
      SBX_HIP(hipMemsetAsync((void*)host[i].rho2, 0, sizeof(T) * (size_t)N * N * N, st));
    SBX_HIP(hipMemsetAsync(host[i].X, 0, sizeof(C2<T>) * x_elems(N), st));
    SBX_HIP(hipMemsetAsync(host[i].C, 0, sizeof(C2<T>) * c_elems(N), st));
    SBX_HIP(hipMemsetAsync(host[i].D, 0, sizeof(C2<T>) * c_elems(N), st));
  }
  hipEvent_t e0, e1;
  SBX_HIP(hipEventCreate(&e0));
  SBX_HIP(hipEventCreate(&e1));
  // fastest of 5 timed repetitions (after 2 untimed) of one launch
  auto time_it = [&](auto&& launch, float& ms_min) -> sbx_status {
    ms_min = 1e30f;
    for (int rep = 0; rep < 7; ++rep) {
      hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, counter, 1);
      SBX_HIP(hipEventRecord(e0, st));
      launch();
      SBX_HIP(hipEventRecord(e1, st));
      SBX_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SBX_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep >= 2) ms_min = std::min(ms_min, ms);
    }
    return SBX_OK;
  };
  // best shape of one line pass (pass 5: the z pass on the plane layout)
  auto tune_pass = [&](int pass, PassShape& pick, float& best) -> sbx_status {
    best = 1e30f;
    pick = PassShape{256, 0, vs[0]};
    for (size_t vi = 0; vi < vs.size(); ++vi)
      for (int nt : nts) {
        if (!shape_ok<T>(nt, vs[vi], N, pass)) continue;
        for (int bpc : bpcs) {
          const PassShape sh{nt, bpc == 0 ? 0 : cus * bpc, vs[vi]};
          float ms = 0.f;
          SBX_TRY(time_it([&] { launch_any<T>(pass, d_solves, N, count, sh, counter, nullptr, tws[vi], st); },
                          ms));
          if (ms < best) {
            best = ms;
            pick = sh;
          }
        }
      }
    return SBX_OK;
  };
  float t5 = 0.f, t3 = 1e30f;
  Tuned five_t, plane_t;
  if (five)
    for (int pass = 0; pass < kPasses; ++pass) {
      float b = 0.f;
      SBX_TRY(tune_pass(pass, five_t.sh[pass], b));
      t5 += b;
    }
  if (plane) {
    plane_t.form = 3;
    float tz = 0.f;
    SBX_TRY(tune_pass(5, plane_t.sh[2], tz));
    t3 = tz;
    const int npin = g_pin_nt.load();
    for (int q : {0, 3}) {
      float best = 1e30f;
      PassShape pick{256, 0, 0};
      const bool pinned = npin && plane_nt_ok<T>(N, npin, q == 3);
      for (int nt : {256, 512, 1024}) {
        if (!plane_nt_ok<T>(N, nt, q == 3) || (pinned && nt != npin)) continue;
        float ms = 0.f;
        SBX_TRY(time_it([&] { launch_plane<T>(q == 3, d_solves, N, count, nt, nullptr, twh, twist, st); }, ms));
        if (ms < best) {
          best = ms;
          pick = PassShape{nt, 0, 0};
        }
      }
      plane_t.sh[q] = pick;
      t3 += best;
    }
    plane_t.sh[1] = plane_t.sh[4] = PassShape{0, 0, 0};
  }
  if (plane && five) {
    // The forms are compared as whole solves, the way a step runs them:
    // the last-level cache is first overwritten (other work of a step
    // streams far more than its 256 MB between two solve sets) and then the
    // inputs are written, as the mass assignment does.  Passes timed alone
    // or back to back find their inputs, intermediates and Green's tables
    // in the caches, which favours the form with more passes.  Repetitions
    // are interleaved so that drifts reach both forms alike: fastest of 10
    // after 2 each.
    const size_t flush_bytes = (size_t)512 << 20;
    void* flush = nullptr;
    if (hipMalloc(&flush, flush_bytes) != hipSuccess) {
      (void)hipGetLastError();
      flush = nullptr;  // compared with warm caches instead
    }
    auto whole = [&](const Tuned& f, float& ms) -> sbx_status {
      if (flush) SBX_HIP(hipMemsetAsync(flush, 0, flush_bytes, st));
      for (int i = 0; i < count; ++i) {
        SBX_HIP(hipMemsetAsync((void*)host[i].rho, 0, sizeof(T) * (size_t)N * N * N, st));
        if (host[i].rho2) SBX_HIP(hipMemsetAsync((void*)host[i].rho2, 0, sizeof(T) * (size_t)N * N * N, st));
      }
      hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, counter, kPasses);
      SBX_HIP(hipEventRecord(e0, st));
      for (int q = 0; q < kPasses; ++q) {
        const bool pq = f.form == 3 && q != 2;
        const C2<T>* tq = pq ? twh : tws[f.sh[q].v == vs[0] || vs.size() == 1 ? 0 : 1];
        run_pass<T>(f.form, q, d_solves, N, count, f.sh[q], counter + q, nullptr, tq, twist, st);
      }
      SBX_HIP(hipEventRecord(e1, st));
      SBX_HIP(hipEventSynchronize(e1));
      SBX_HIP(hipEventElapsedTime(&ms, e0, e1));
      return SBX_OK;
    };
    t5 = t3 = 1e30f;
    sbx_status rc = SBX_OK;
    for (int rep = 0; rep < 12 && rc == SBX_OK; ++rep) {
      float a = 0.f, b = 0.f;
      if ((rc = whole(five_t, a)) == SBX_OK) rc = whole(plane_t, b);
      if (rep >= 2) {
        t5 = std::min(t5, a);
        t3 = std::min(t3, b);
      }
    }
    if (flush) (void)hipFree(flush);
    SBX_TRY(rc);
  }
  // Within 5% (the spread of these timings from one process to the next)
  // the form that moves fewer bytes wins: the plane form, whose margin
  // inside a step has been larger than in this isolated comparison.
  out = (plane && (!five || t3 < 1.05f * t5)) ? plane_t : five_t;
  out.ms5 = five ? t5 : 0.f;
  out.ms3 = plane ? t3 : 0.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return SBX_OK;
}

template <typename T>
sbx_status plan_create(SolvePlan<T>& p, const SolveDesc<T>* descs, int n, hipStream_t st) {
  plan_destroy(p);
  if (n <= 0) return SBX_OK;
  for (int i = 0; i < n; ++i) {
    const int N = descs[i].N;
    if (N < 8 || N > 256 || (N & (N - 1))) {
      set_error("grid size must be a power of two in 8..256");
      return SBX_EINVAL;
    }
  }
  // solves grouped by grid size (stable), one launch per group and pass
  p.host.assign(descs, descs + n);
  std::stable_sort(p.host.begin(), p.host.end(),
                   [](const SolveDesc<T>& a, const SolveDesc<T>& b) { return a.N < b.N; });
  p.nsolves = n;
  if (hipMalloc(&p.d_solves, sizeof(SolveDesc<T>) * n) != hipSuccess ||
      hipMalloc(&p.d_counter, sizeof(int) * kPasses * kMaxGroups) != hipSuccess) {
    (void)hipGetLastError();
    plan_destroy(p);
    set_error("out of device memory (solve plan)");
    return SBX_ENOMEM;
  }
  SBX_HIP(hipMemcpy(p.d_solves, p.host.data(), sizeof(SolveDesc<T>) * n, hipMemcpyHostToDevice));
  p.ngroups = 0;
  for (int i = 0; i < n;) {
    int j = i;
    while (j < n && p.host[j].N == p.host[i].N) ++j;
    if (p.ngroups == kMaxGroups) {
      set_error("too many distinct grid sizes in one plan");
      return SBX_EINVAL;
    }
    SolveGroup& g = p.groups[p.ngroups++];
    g.first = i;
    g.count = j - i;
    g.N = p.host[i].N;
    i = j;
  }
  if (p.ngroups > 1) {
    bool ok = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) == hipSuccess;
    for (int gi = 1; ok && gi < p.ngroups; ++gi)
      ok = hipStreamCreateWithFlags(&p.side[gi], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&p.join[gi], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      plan_destroy(p);
      set_error("stream or event creation failed (solve plan)");
      return SBX_EDEVICE;
    }
  }
  for (int gi = 0; gi < p.ngroups; ++gi) {
    SolveGroup& g = p.groups[gi];
    Tuned a;
    const TuneKey key = key_now((int)sizeof(T), g.N, g.count);
    if (!tune_lookup(key, a)) {
      SBX_TRY(tune_group<T>(p.d_solves + g.first, p.host.data() + g.first, g.N, g.count,
                            p.d_counter, st, a));
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune.push_back({key, a});
    }
    g.form = a.form;
    if (g.form == 3 && !plane_ok<T>(g.N)) {
      set_error("internal: plane-fused form chosen for a size without one");
      return SBX_EINVAL;
    }
    for (int q = 0; q < kPasses; ++q) {
      g.shape[q] = a.sh[q];
      g.tw[q] = nullptr;
      if (g.form == 3 && (q == 1 || q == 4)) continue;
      // the plane passes transform lines of N (16 values per lane)
      const bool pq = g.form == 3 && q != 2;
      const C2<T>* tw = pq ? twiddles<T>(g.N, 16, st) : twiddles<T>(2 * g.N, a.sh[q].v, st);
      if (!tw) {
        set_error("twiddle table allocation failed");
        return SBX_ENOMEM;
      }
      g.tw[q] = (const void*)tw;
    }
    g.twist = nullptr;
    if (g.form == 3 && (!(g.twist = (const void*)twist_table<T>(g.N, st)) || !plane_tables<T>(g.N, st))) {
      set_error("twiddle table allocation failed");
      return SBX_ENOMEM;
    }
  }
  // work counters start at zero; every pass then clears its predecessor's
  SBX_HIP(hipMemsetAsync(p.d_counter, 0, sizeof(int) * kPasses * kMaxGroups, st));
  SBX_HIP(hipStreamSynchronize(st));
  return SBX_OK;
}

template <typename T>
sbx_status plan_run_pass(const SolvePlan<T>& p, int q, int group, hipStream_t st) {
  const SolveGroup& g = p.groups[group];
  run_pass<T>(g.form, q, p.d_solves + g.first, g.N, g.count, g.shape[q], p.d_counter + q * kMaxGroups + group,
              p.d_counter + ((q + kPasses - 1) % kPasses) * kMaxGroups + group, (const C2<T>*)g.tw[q],
              (const C2<T>*)g.twist, st);
  return SBX_OK;
}

template <typename T>
sbx_status plan_run(const SolvePlan<T>& p, hipStream_t st, Recorder* rec) {
  if (p.nsolves == 0) return SBX_OK;
  Recorder none;
  Recorder& r = rec ? *rec : none;
  static const int marks[kPasses] = {PH_FWD_X, PH_FWD_Y, PH_ZPASS, PH_INV_Y, PH_INV_X};
  if (p.ngroups == 1) {
    for (int q = 0; q < kPasses; ++q) {
      SBX_TRY(plan_run_pass<T>(p, q, 0, st));
      r.mark(marks[q], st);
    }
  } else {
    // independent size groups: group 0 on the caller's stream, the others
    // on their own streams between a fork and a join
    SBX_HIP(hipEventRecord(p.fork, st));
    for (int gi = 1; gi < p.ngroups; ++gi) SBX_HIP(hipStreamWaitEvent(p.side[gi], p.fork, 0));
    for (int gi = 0; gi < p.ngroups; ++gi)
      for (int q = 0; q < kPasses; ++q) SBX_TRY(plan_run_pass<T>(p, q, gi, gi == 0 ? st : p.side[gi]));
    for (int gi = 1; gi < p.ngroups; ++gi) {
      SBX_HIP(hipEventRecord(p.join[gi], p.side[gi]));
      SBX_HIP(hipStreamWaitEvent(st, p.join[gi], 0));
    }
    for (int q = 0; q < kPasses; ++q) r.mark(marks[q], st);
  }
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status prepare_twiddles(int N, hipStream_t st) {
  for (int v : {16, 32})
    if (!twiddles<T>(2 * N, v, st)) {
      set_error("twiddle table allocation failed");
      return SBX_ENOMEM;
    }
  if (plane_ok<T>(N) && !plane_tables<T>(N, st)) {
    set_error("twiddle table allocation failed");
    return SBX_ENOMEM;
  }
  return SBX_OK;
}

template <typename T>
sbx_status run_solves_noalloc(const SolveDesc<T>* d_solves, int nsolves, int N, int* d_counter,
                              hipStream_t st) {
  Tuned a;
  if (!tune_lookup(key_now((int)sizeof(T), N, nsolves), a))
    for (auto& sh : a.sh) sh = PassShape{256, 0, 0};
  const C2<T>* tw[kPasses] = {};
  const C2<T>* twist = a.form == 3 ? twist_table<T>(N, st, false) : nullptr;
  if (a.form == 3 && N == 128 && PH<T, 128>::fits && !twiddles<T>(N / 2, 16, st, false)) {
    set_error("no twiddle table for this grid size on this device (create a plan first)");
    return SBX_ESTATE;
  }
  for (int q = 0; q < kPasses; ++q) {
    if (a.form == 3 && (q == 1 || q == 4)) continue;
    tw[q] = (a.form == 3 && q != 2) ? twiddles<T>(N, 16, st, false) : twiddles<T>(2 * N, a.sh[q].v, st, false);
    if (!tw[q] || (a.form == 3 && !twist)) {
      set_error("no twiddle table for this grid size on this device (create a plan first)");
      return SBX_ESTATE;
    }
  }
  for (int q = 0; q < kPasses; ++q)
    run_pass<T>(a.form, q, d_solves, N, nsolves, a.sh[q], d_counter + q, d_counter + (q + kPasses - 1) % kPasses,
                tw[q], twist, st);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template sbx_status prepare_twiddles<float>(int, hipStream_t);
template sbx_status prepare_twiddles<double>(int, hipStream_t);
template sbx_status run_solves_noalloc<float>(const SolveDesc<float>*, int, int, int*, hipStream_t);
template sbx_status run_solves_noalloc<double>(const SolveDesc<double>*, int, int, int*, hipStream_t);

template <typename T>
void plan_destroy(SolvePlan<T>& p) {
  if (p.d_solves) (void)hipFree(p.d_solves);
  if (p.d_counter) (void)hipFree(p.d_counter);
  for (int gi = 0; gi < kMaxGroups; ++gi) {
    if (p.side[gi]) (void)hipStreamDestroy(p.side[gi]);
    if (p.join[gi]) (void)hipEventDestroy(p.join[gi]);
  }
  if (p.fork) (void)hipEventDestroy(p.fork);
  p = SolvePlan<T>();
}

template sbx_status plan_create<float>(SolvePlan<float>&, const SolveDesc<float>*, int, hipStream_t);
template sbx_status plan_create<double>(SolvePlan<double>&, const SolveDesc<double>*, int, hipStream_t);
template sbx_status plan_run<float>(const SolvePlan<float>&, hipStream_t, Recorder*);
template sbx_status plan_run<double>(const SolvePlan<double>&, hipStream_t, Recorder*);
template sbx_status plan_run_pass<float>(const SolvePlan<float>&, int, int, hipStream_t);
template sbx_status plan_run_pass<double>(const SolvePlan<double>&, int, int, hipStream_t);
template void plan_destroy<float>(SolvePlan<float>&);
template void plan_destroy<double>(SolvePlan<double>&);

// ---------------------------------------------------- Green's table (FP64) --
// H of Eq. 2 on the doubled grid, mirrored by Eq. 5: F[z][y][x] with lags
// fold(x) * l, fold(y) * l, fold(z) * lz, fold(k) = min(k, 2N - k).
__global__ void k_green_fill(C2<double>* F, int N, double l, double lz, double h0) {
  const int L = 2 * N;
  const size_t n = (size_t)L * L * L;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((size_t)L * L));
    const int fx = x <= N ? x : L - x, fy = y <= N ? y : L - y, fz = z <= N ? z : L - z;
    double h;
    if (fx == 0 && fy == 0 && fz == 0) {
      h = h0;
    } else {
      const double X = (double)fx * l, Y = (double)fy * l, Z = (double)fz * lz;
      h = 1.0 / sqrt(X * X + Y * Y + Z * Z);
    }
    F[i] = C2<double>{h, 0.0};
  }
}

// In-place complex FFT of every line of F along one axis: W lines per block
// staged in LDS, each transformed by TL threads of one wave.
template <int L>
struct GreenTile {
  static constexpr int TL = Line<double, L, kDefV<double, L>>::TL, P = L + L / 16 + 1, NT = 256;
  static constexpr int fit(int w) {
    return (w > 1 && w * P * (int)sizeof(C2<double>) > kLdsCap) ? fit(w / 2) : w;
  }
  static constexpr int W = fit(NT / TL < L ? NT / TL : L);
};

template <int L, int AXIS>
__global__ void __launch_bounds__(256)
    k_c2c_axis(C2<double>* F, const C2<double>* __restrict__ tw) {
  using K = GreenTile<L>;
  constexpr int W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<double> s[W * P];
  const int o = blockIdx.x / (L / W), i0 = (blockIdx.x % (L / W)) * W;
  const size_t es = AXIS == 0 ? 1 : (AXIS == 1 ? (size_t)L : (size_t)L * L);
  const size_t ws = AXIS == 0 ? (size_t)L : 1;
  C2<double>* base = F + (AXIS == 0 ? (size_t)o * L * L + (size_t)i0 * L
                                    : (AXIS == 1 ? (size_t)o * L * L : (size_t)o * L) + i0);
  for (int i = threadIdx.x; i < W * L; i += NT) {
    const int e = AXIS == 0 ? i % L : i / W, w = AXIS == 0 ? i / L : i % W;
    s[w * P + pad(e)] = base[e * es + w * ws];
  }
  __syncthreads();
  if ((int)threadIdx.x < W * TL)
    line_fwd_lds<double, L, kDefV<double, L>>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
  __syncthreads();
  for (int i = threadIdx.x; i < W * L; i += NT) {
    const int e = AXIS == 0 ? i % L : i / W, w = AXIS == 0 ? i / L : i % W;
    base[e * es + w * ws] = s[w * P + pad(e)];
  }
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_green_absmax(const C2<double>* F, size_t n, unsigned long long* out) {
  double mr = 0.0, mi = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    mr = fmax(mr, fabs(F[i].re));
    mi = fmax(mi, fabs(F[i].im));
  }
  atomic_max_pos(out, mr);
  atomic_max_pos(out + 1, mi);
}

template <typename T>
__global__ void k_green_fold(const C2<double>* F, T* H, int N, double scale) {
  const int L = 2 * N, M = N + 1;
  const size_t n = (size_t)M * M * M;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % M), ky = (int)((i / M) % M), kx = (int)(i / ((size_t)M * M));
    H[i] = (T)(scale * F[((size_t)kz * L + ky) * L + kx].re);
  }
}

template <int L>
static sbx_status green_fft(C2<double>* F, hipStream_t st) {
  using K = GreenTile<L>;
  const C2<double>* tw = twiddles<double>(L, 0, st);
  if (!tw) {
    set_error("twiddle table allocation failed");
    return SBX_ENOMEM;
  }
  const dim3 g(L * (L / K::W)), b(256);
  hipLaunchKernelGGL((k_c2c_axis<L, 0>), g, b, 0, st, F, tw);
  hipLaunchKernelGGL((k_c2c_axis<L, 1>), g, b, 0, st, F, tw);
  hipLaunchKernelGGL((k_c2c_axis<L, 2>), g, b, 0, st, F, tw);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

// Mean of 1/r over a cell of sides (lx, ly, lz) about its centre: eight
// octants of the integral of 1/r over a box [0,a]x[0,b]x[0,c] taken from a
// corner (the potential of a uniform rectangular prism at its corner).
static double cell_mean_inv_r(double lx, double ly, double lz) {
  const double a = 0.5 * lx, b = 0.5 * ly, c = 0.5 * lz;
  const double r = std::sqrt(a * a + b * b + c * c);
  const double f = b * c * std::asinh(a / std::hypot(b, c)) + a * c * std::asinh(b / std::hypot(a, c)) +
                   a * b * std::asinh(c / std::hypot(a, b)) - 0.5 * a * a * std::atan(b * c / (a * r)) -
                   0.5 * b * b * std::atan(a * c / (b * r)) - 0.5 * c * c * std::atan(a * b / (c * r));
  return 8.0 * f / (lx * ly * lz);
}

// Largest admissible max|Im| / max|Re| of the FP64 transform of the mirrored
// Green's function: Eq. 5 makes it real, so only rounding may remain.
constexpr double kGreenImagTol = 1e-10;

template <typename T>
sbx_status build_green(int N, double l, double lz, double G, int h0_mode, T* H, double* rel_imag,
                       hipStream_t st) {
  const int L = 2 * N;
  const size_t n = (size_t)L * L * L;
  C2<double>* F = nullptr;
  unsigned long long* mx = nullptr;
  if (hipMalloc(&F, n * sizeof(C2<double>)) != hipSuccess) {
    set_error("Green's table work grid: out of device memory");
    return SBX_ENOMEM;
  }
  if (hipMalloc(&mx, 2 * sizeof(unsigned long long)) != hipSuccess) {
    (void)hipFree(F);
    set_error("out of device memory");
    return SBX_ENOMEM;
  }
  const double h0 = h0_mode == 2 ? 0.0 : (h0_mode == 1 ? cell_mean_inv_r(l, l, lz) : 1.0 / l);
  sbx_status rc = SBX_OK;
  hipLaunchKernelGGL(k_green_fill, dim3(2048), dim3(256), 0, st, F, N, l, lz, h0);
  switch (N) {
    case 8: rc = green_fft<16>(F, st); break;
    case 16: rc = green_fft<32>(F, st); break;
    case 32: rc = green_fft<64>(F, st); break;
    case 64: rc = green_fft<128>(F, st); break;
    case 128: rc = green_fft<256>(F, st); break;
    case 256: rc = green_fft<512>(F, st); break;
    default: set_error("grid size must be a power of two in 8..256"); rc = SBX_EINVAL;
  }
  if (rc == SBX_OK) {
    const double scale = G / ((double)L * L * L);
    unsigned long long host[2] = {0, 0};
    if (hipMemsetAsync(mx, 0, 2 * sizeof(unsigned long long), st) != hipSuccess) rc = SBX_EDEVICE;
    hipLaunchKernelGGL(k_green_absmax, dim3(1024), dim3(256), 0, st, F, n, mx);
    hipLaunchKernelGGL((k_green_fold<T>), dim3(2048), dim3(256), 0, st, F, H, N, scale);
    if (hipMemcpyAsync(host, mx, sizeof(host), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error(std::string("Green's table build: ") + hipGetErrorString(hipGetLastError()));
      rc = SBX_EDEVICE;
    } else {
      double re, im;
      memcpy(&re, &host[0], 8);
      memcpy(&im, &host[1], 8);
      const double ri = re > 0 ? im / re : 1.0;
      if (rel_imag) *rel_imag = ri;
      if (!(ri <= kGreenImagTol)) {
        set_error("transformed Green's function not real to rounding (max|Im|/max|Re| = " +
                  std::to_string(ri) + "): the mirror symmetry of Eq. 5 is broken");
        rc = SBX_EPARITY;
      }
    }
  }
  (void)hipFree(mx);
  (void)hipFree(F);
  return rc;
}

template sbx_status build_green<float>(int, double, double, double, int, float*, double*, hipStream_t);
template sbx_status build_green<double>(int, double, double, double, int, double*, double*,
                                        hipStream_t);

}  // namespace sbx
