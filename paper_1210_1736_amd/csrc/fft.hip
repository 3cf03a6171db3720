// Batched pruned 3D FFT convolution with the isolated-boundary Green's
// function (Eqs. 3-5 of the method) and the FP64 Green's-table build.
//
// Each block holds W lines of length L = 2N in LDS and runs a Stockham
// autosort FFT on them: a radix-16 pass (one 16-point DFT in registers per
// thread), then the remaining radix (2, 4, 8 or 16) with twiddles from a
// table.  Global loads and stores are arranged so that consecutive threads
// touch consecutive addresses: along the line when the line is contiguous,
// across the W lines of a tile when it is strided.
#include <cstring>
#include <mutex>

#include "fft.h"

namespace sbx {

__device__ __forceinline__ int pad(int e) { return e + (e >> 4); }

template <typename T, int L>
struct Cfg {
  static constexpr int N = L / 2;
  static constexpr int TL = L / 16;                  // threads per line
  static constexpr int P = L + L / 16 + 1;           // LDS pitch of one line
  static constexpr int WCAP = (40960 / (P * (int)sizeof(C2<T>))) >= 16 ? 16
                              : (40960 / (P * (int)sizeof(C2<T>))) >= 8 ? 8 : 4;
  static constexpr int WMAX = sizeof(T) == 4 ? 16 : 8;
  static constexpr int W0 = WCAP < WMAX ? WCAP : WMAX;
  static constexpr int W = N < W0 ? N : W0;          // lines per block
  static constexpr int NT = W * TL;                  // threads per block
};

// ------------------------------------------------------------- Stockham ---
// One pass of radix R with stride NS over a line in LDS (in place).
template <typename T, int L, int R, int NS, bool INV, bool PIN, bool POUT>
__device__ __forceinline__ void st_pass(C2<T>* line, int t, const C2<T>* __restrict__ tw) {
  constexpr int TL = L / 16, NB = L / R, BPT = NB / TL;
  C2<T> v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = t + b * TL;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (PIN && r >= R / 2) v[b][r] = C2<T>{(T)0, (T)0};
      else v[b][r] = line[pad(j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = t + b * TL;
    const int k = j & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C2<T> w = tw[(r - 1) * NS + k];
        if (INV) w.im = -w.im;
        v[b][r] = cmul(v[b][r], w);
      }
    }
    dftR<R, INV>(v[b]);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (POUT && r >= R / 2) continue;
      line[pad(base + r * NS)] = v[b][r];
    }
  }
  __syncthreads();
}

// Full length-L transform of one line by the TL threads t = 0..TL-1.
// PIN: input is zero in [L/2, L); POUT: only [0, L/2) of the output is kept.
template <typename T, int L, bool INV, bool PIN, bool POUT>
__device__ __forceinline__ void fft_line(C2<T>* line, int t, const C2<T>* __restrict__ tw) {
  if constexpr (L == 16) {
    st_pass<T, L, 16, 1, INV, PIN, POUT>(line, t, tw);
  } else if constexpr (L == 32) {
    st_pass<T, L, 16, 1, INV, PIN, false>(line, t, tw);
    st_pass<T, L, 2, 16, INV, false, POUT>(line, t, tw);
  } else if constexpr (L == 64) {
    st_pass<T, L, 16, 1, INV, PIN, false>(line, t, tw);
    st_pass<T, L, 4, 16, INV, false, POUT>(line, t, tw);
  } else if constexpr (L == 128) {
    st_pass<T, L, 16, 1, INV, PIN, false>(line, t, tw);
    st_pass<T, L, 8, 16, INV, false, POUT>(line, t, tw);
  } else if constexpr (L == 256) {
    st_pass<T, L, 16, 1, INV, PIN, false>(line, t, tw);
    st_pass<T, L, 16, 16, INV, false, POUT>(line, t, tw);
  } else {
    static_assert(L == 512, "L in 16..512");
    st_pass<T, L, 16, 1, INV, PIN, false>(line, t, tw);
    st_pass<T, L, 16, 16, INV, false, false>(line, t, tw);
    st_pass<T, L, 2, 256, INV, false, POUT>(line, t, tw + 240);
  }
}

// Twiddle table for length L: for every pass after the first, entries
// (r-1)*NS + k = exp(-2 pi i k r / (NS R)), r = 1..R-1, k = 0..NS-1.
static int tw_len(int L) {
  switch (L) {
    case 16: return 1;
    case 32: return 16;
    case 64: return 48;
    case 128: return 112;
    case 256: return 240;
    default: return 496;
  }
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

template <typename T>
const C2<T>* twiddles(int L, hipStream_t st) {
  static std::mutex mu;
  static C2<T>* cache[64][10] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  std::lock_guard<std::mutex> g(mu);
  if (cache[dev][lg]) return cache[dev][lg];
  C2<T>* p = nullptr;
  if (hipMalloc(&p, sizeof(C2<T>) * tw_len(L)) != hipSuccess) return nullptr;
  struct PassRN { int R, NS, off; };
  PassRN ps[2] = {{0, 0, 0}, {0, 0, 0}};
  int np = 0;
  switch (L) {
    case 32: ps[0] = {2, 16, 0}; np = 1; break;
    case 64: ps[0] = {4, 16, 0}; np = 1; break;
    case 128: ps[0] = {8, 16, 0}; np = 1; break;
    case 256: ps[0] = {16, 16, 0}; np = 1; break;
    case 512: ps[0] = {16, 16, 0}; ps[1] = {2, 256, 240}; np = 2; break;
    default: break;
  }
  for (int i = 0; i < np; ++i) {
    const int n = (ps[i].R - 1) * ps[i].NS;
    hipLaunchKernelGGL(k_twiddle<T>, dim3((n + 255) / 256), dim3(256), 0, st, p + ps[i].off,
                       ps[i].R, ps[i].NS);
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(p);
    return nullptr;
  }
  cache[dev][lg] = p;
  return p;
}

template const C2<float>* twiddles<float>(int, hipStream_t);
template const C2<double>* twiddles<double>(int, hipStream_t);

// ------------------------------------------------------------ the passes ---
// fwd_x: tile = W consecutive y at one z; real input, x < N.
template <typename T, int L>
__global__ void __launch_bounds__((Cfg<T, L>::NT))
    k_fwd_x(const SolveBatch<T> desc, const C2<T>* __restrict__ tw) {
  using K = Cfg<T, L>;
  constexpr int N = K::N, W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<T> s[W * P];
  const SolveDesc<T>& d = desc.d[blockIdx.y];
  const int z = blockIdx.x / (N / W), y0 = (blockIdx.x % (N / W)) * W;
  const T* __restrict__ src = d.rho + ((size_t)z * N + y0) * N;
  for (int i = threadIdx.x; i < W * N; i += NT) {
    const int w = i / N, e = i - w * N;
    s[w * P + pad(e)] = C2<T>{src[i], (T)0};
  }
  __syncthreads();
  fft_line<T, L, false, true, false>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
  C2<T>* __restrict__ dst = d.X + (size_t)z * N + y0;
  for (int i = threadIdx.x; i < W * (N + 1); i += NT) {
    const int e = i / W, w = i - e * W;
    dst[(size_t)e * N * N + w] = s[w * P + pad(e)];
  }
}

// fwd_y: tile = W consecutive z at one kx; input y < N contiguous.
template <typename T, int L>
__global__ void __launch_bounds__((Cfg<T, L>::NT))
    k_fwd_y(const SolveBatch<T> desc, const C2<T>* __restrict__ tw) {
  using K = Cfg<T, L>;
  constexpr int N = K::N, W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<T> s[W * P];
  const SolveDesc<T>& d = desc.d[blockIdx.y];
  const int kx = blockIdx.x / (N / W), z0 = (blockIdx.x % (N / W)) * W;
  const C2<T>* __restrict__ src = d.X + ((size_t)kx * N + z0) * N;
  for (int i = threadIdx.x; i < W * N; i += NT) {
    const int w = i / N, e = i - w * N;
    s[w * P + pad(e)] = src[i];
  }
  __syncthreads();
  fft_line<T, L, false, true, false>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
  C2<T>* __restrict__ dst = d.C + (size_t)kx * L * N + z0;
  for (int i = threadIdx.x; i < W * L; i += NT) {
    const int e = i / W, w = i - e * W;
    dst[(size_t)e * N + w] = s[w * P + pad(e)];
  }
}

// zpass: tile = W consecutive ky at one kx; forward z, times Hhat, inverse z.
template <typename T, int L>
__global__ void __launch_bounds__((Cfg<T, L>::NT))
    k_zpass(const SolveBatch<T> desc, const C2<T>* __restrict__ tw) {
  using K = Cfg<T, L>;
  constexpr int N = K::N, W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<T> s[W * P];
  const SolveDesc<T>& d = desc.d[blockIdx.y];
  const int kx = blockIdx.x / (L / W), ky0 = (blockIdx.x % (L / W)) * W;
  C2<T>* __restrict__ base = d.C + ((size_t)kx * L + ky0) * N;
  for (int i = threadIdx.x; i < W * N; i += NT) {
    const int w = i / N, e = i - w * N;
    s[w * P + pad(e)] = base[i];
  }
  __syncthreads();
  C2<T>* line = s + (threadIdx.x / TL) * P;
  fft_line<T, L, false, true, false>(line, threadIdx.x % TL, tw);
  const T* __restrict__ H = d.H + (size_t)kx * (N + 1) * (N + 1);
  for (int i = threadIdx.x; i < W * L; i += NT) {
    const int w = i / L, e = i - w * L;
    const int ky = ky0 + w;
    const int fy = ky <= N ? ky : L - ky;
    const int fz = e <= N ? e : L - e;
    const T h = H[fy * (N + 1) + fz];
    C2<T>& c = s[w * P + pad(e)];
    c = cscale(c, h);
  }
  __syncthreads();
  fft_line<T, L, true, false, true>(line, threadIdx.x % TL, tw);
  for (int i = threadIdx.x; i < W * N; i += NT) {
    const int w = i / N, e = i - w * N;
    base[i] = s[w * P + pad(e)];
  }
}

// inv_y: tile = W consecutive z at one kx; ky strided by N; keep y < N.
template <typename T, int L>
__global__ void __launch_bounds__((Cfg<T, L>::NT))
    k_inv_y(const SolveBatch<T> desc, const C2<T>* __restrict__ tw) {
  using K = Cfg<T, L>;
  constexpr int N = K::N, W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<T> s[W * P];
  const SolveDesc<T>& d = desc.d[blockIdx.y];
  const int kx = blockIdx.x / (N / W), z0 = (blockIdx.x % (N / W)) * W;
  const C2<T>* __restrict__ src = d.C + (size_t)kx * L * N + z0;
  for (int i = threadIdx.x; i < W * L; i += NT) {
    const int e = i / W, w = i - e * W;
    s[w * P + pad(e)] = src[(size_t)e * N + w];
  }
  __syncthreads();
  fft_line<T, L, true, false, true>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
  C2<T>* __restrict__ dst = d.X + ((size_t)kx * N + z0) * N;
  for (int i = threadIdx.x; i < W * N; i += NT) {
    const int w = i / N, e = i - w * N;
    dst[i] = s[w * P + pad(e)];
  }
}

// inv_x: tile = W consecutive y at one z; kx <= N strided by N*N, the rest
// of the line by Hermitian symmetry; real output x < N.
template <typename T, int L>
__global__ void __launch_bounds__((Cfg<T, L>::NT))
    k_inv_x(const SolveBatch<T> desc, const C2<T>* __restrict__ tw) {
  using K = Cfg<T, L>;
  constexpr int N = K::N, W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<T> s[W * P];
  const SolveDesc<T>& d = desc.d[blockIdx.y];
  const int z = blockIdx.x / (N / W), y0 = (blockIdx.x % (N / W)) * W;
  const C2<T>* __restrict__ src = d.X + (size_t)z * N + y0;
  for (int i = threadIdx.x; i < W * (N + 1); i += NT) {
    const int e = i / W, w = i - e * W;
    const C2<T> v = src[(size_t)e * N * N + w];
    s[w * P + pad(e)] = v;
    if (e >= 1 && e < N) s[w * P + pad(L - e)] = conjc(v);
  }
  __syncthreads();
  fft_line<T, L, true, false, true>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
  T* __restrict__ dst = d.phi + ((size_t)z * N + y0) * N;
  for (int i = threadIdx.x; i < W * N; i += NT) {
    const int w = i / N, e = i - w * N;
    dst[i] = s[w * P + pad(e)].re;
  }
}

template <typename T, int L>
static sbx_status launch_solve(int nsolves, const SolveBatch<T>& desc, hipStream_t st,
                               Recorder* rec) {
  using K = Cfg<T, L>;
  constexpr int N = K::N, W = K::W;
  const C2<T>* tw = twiddles<T>(L, st);
  if (!tw) {
    set_error("twiddle table allocation failed");
    return SBX_ENOMEM;
  }
  const dim3 b(K::NT);
  Recorder none;
  Recorder& r = rec ? *rec : none;
  hipLaunchKernelGGL((k_fwd_x<T, L>), dim3(N * (N / W), nsolves), b, 0, st, desc, tw);
  r.mark(PH_FWD_X, st);
  hipLaunchKernelGGL((k_fwd_y<T, L>), dim3((N + 1) * (N / W), nsolves), b, 0, st, desc, tw);
  r.mark(PH_FWD_Y, st);
  hipLaunchKernelGGL((k_zpass<T, L>), dim3((N + 1) * (L / W), nsolves), b, 0, st, desc, tw);
  r.mark(PH_ZPASS, st);
  hipLaunchKernelGGL((k_inv_y<T, L>), dim3((N + 1) * (N / W), nsolves), b, 0, st, desc, tw);
  r.mark(PH_INV_Y, st);
  hipLaunchKernelGGL((k_inv_x<T, L>), dim3(N * (N / W), nsolves), b, 0, st, desc, tw);
  r.mark(PH_INV_X, st);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status solve_batch(int N, int nsolves, const SolveBatch<T>& desc, hipStream_t st,
                       Recorder* rec) {
  if (nsolves <= 0) return SBX_OK;
  if (nsolves > kMaxBatch) {
    set_error("too many solves in one batch");
    return SBX_EINVAL;
  }
  switch (N) {
    case 8: return launch_solve<T, 16>(nsolves, desc, st, rec);
    case 16: return launch_solve<T, 32>(nsolves, desc, st, rec);
    case 32: return launch_solve<T, 64>(nsolves, desc, st, rec);
    case 64: return launch_solve<T, 128>(nsolves, desc, st, rec);
    case 128: return launch_solve<T, 256>(nsolves, desc, st, rec);
    case 256: return launch_solve<T, 512>(nsolves, desc, st, rec);
    default: set_error("grid size must be a power of two in 8..256"); return SBX_EINVAL;
  }
}

template sbx_status solve_batch<float>(int, int, const SolveBatch<float>&, hipStream_t, Recorder*);
template sbx_status solve_batch<double>(int, int, const SolveBatch<double>&, hipStream_t, Recorder*);

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

// In-place complex FFT of every line of F along one axis.
template <int L, int AXIS>
__global__ void __launch_bounds__((Cfg<double, L>::NT))
    k_c2c_axis(C2<double>* F, const C2<double>* __restrict__ tw) {
  using K = Cfg<double, L>;
  constexpr int W = K::W, P = K::P, NT = K::NT, TL = K::TL;
  __shared__ C2<double> s[W * P];
  const int o = blockIdx.x / (L / W), i0 = (blockIdx.x % (L / W)) * W;
  if constexpr (AXIS == 0) {
    C2<double>* base = F + ((size_t)o * L + i0) * L;
    for (int i = threadIdx.x; i < W * L; i += NT) {
      const int w = i / L, e = i - w * L;
      s[w * P + pad(e)] = base[i];
    }
    __syncthreads();
    fft_line<double, L, false, false, false>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
    for (int i = threadIdx.x; i < W * L; i += NT) {
      const int w = i / L, e = i - w * L;
      base[i] = s[w * P + pad(e)];
    }
  } else {
    const size_t es = AXIS == 1 ? (size_t)L : (size_t)L * L;
    C2<double>* base = F + (AXIS == 1 ? (size_t)o * L * L : (size_t)o * L) + i0;
    for (int i = threadIdx.x; i < W * L; i += NT) {
      const int e = i / W, w = i - e * W;
      s[w * P + pad(e)] = base[e * es + w];
    }
    __syncthreads();
    fft_line<double, L, false, false, false>(s + (threadIdx.x / TL) * P, threadIdx.x % TL, tw);
    for (int i = threadIdx.x; i < W * L; i += NT) {
      const int e = i / W, w = i - e * W;
      base[e * es + w] = s[w * P + pad(e)];
    }
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
  using K = Cfg<double, L>;
  const C2<double>* tw = twiddles<double>(L, st);
  if (!tw) {
    set_error("twiddle table allocation failed");
    return SBX_ENOMEM;
  }
  const dim3 g(L * (L / K::W)), b(K::NT);
  hipLaunchKernelGGL((k_c2c_axis<L, 0>), g, b, 0, st, F, tw);
  hipLaunchKernelGGL((k_c2c_axis<L, 1>), g, b, 0, st, F, tw);
  hipLaunchKernelGGL((k_c2c_axis<L, 2>), g, b, 0, st, F, tw);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

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
  const double h0 = h0_mode == 2 ? 0.0 : 1.0 / l;
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
    } else if (rel_imag) {
      double re, im;
      memcpy(&re, &host[0], 8);
      memcpy(&im, &host[1], 8);
      *rel_imag = re > 0 ? im / re : 0.0;
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
