// Particle-side kernels: loss test and centre of mass, classification and
// nearest-grid-point mass assignment, the Eq. 8 force with the grid-selection
// rule fused with the leapfrog kick and drift (Eq. 6), the FP64 diagnostic
// reductions and the cell sort.  Every kernel serves a set of instances
// through a device table (see particles.h).
//
// Cell indices and classes are integers decided by float64 arithmetic with
// every operation rounded separately (no fused multiply-add), so that any
// other implementation following the same formulas gets identical integers.
#include <type_traits>

#include "particles.h"
#include "scan.h"

namespace sbx {

template <typename T>
__device__ __forceinline__ void atomic_add_g(gp<T> p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ cell index --
// Eq. 7: a = [gamma (x - c) + N/2], nearest integer = floor(u + 0.5).
__device__ __forceinline__ int ngp_cell(double x, double c, double gamma, double half) {
#pragma clang fp contract(off)
  const double d = x - c;
  double u = d * gamma;
  u = u + half;
  const double f = floor(u + 0.5);
  // keep the integer conversion defined far outside the grid (and for NaN)
  if (!(f >= -1073741824.0)) return -1073741824;
  if (f > 1073741824.0) return 1073741824;
  return (int)f;
}

// (dx^2 + dy^2) + (dz/q)^2, each operation rounded
__device__ __forceinline__ double sph_r2(double dx, double dy, double dz, double inv_q) {
#pragma clang fp contract(off)
  const double dzq = dz * inv_q;
  const double a = dx * dx;
  const double b = dy * dy;
  const double c = dzq * dzq;
  return (a + b) + c;
}

__device__ __forceinline__ bool usable(const int* i, int N) {
  return i[0] >= 2 && i[0] <= N - 3 && i[1] >= 2 && i[1] <= N - 3 && i[2] >= 2 && i[2] <= N - 3;
}

__device__ __forceinline__ void cell3(const LevelDev& L, const double* c, double x, double y,
                                      double z, int* i) {
  i[0] = ngp_cell(x, c[0], L.gx, L.half);
  i[1] = ngp_cell(y, c[1], L.gx, L.half);
  i[2] = ngp_cell(z, c[2], L.gz, L.half);
}

struct Classified {
  int cls;         // sbx_class
  int idx[3][3];   // cell per level
};

// Class relative to one galaxy's grids (Sec. 2.1): core (inside R1, usable on
// all levels), ring (inside R2, usable on middle and outer), outer (usable on
// the global grid), else lost.
__device__ __forceinline__ void classify(const HierDev& h, const double* c, double x, double y,
                                         double z, Classified& o) {
  if (h.n_levels == 1) {
    cell3(h.lv[0], c, x, y, z, o.idx[0]);
    o.cls = usable(o.idx[0], h.lv[0].N) ? SBX_OUTER : SBX_LOST;
    return;
  }
  cell3(h.lv[0], c, x, y, z, o.idx[0]);
  cell3(h.lv[1], c, x, y, z, o.idx[1]);
  cell3(h.lv[2], h.outer_c, x, y, z, o.idx[2]);
  const bool ok1 = usable(o.idx[0], h.lv[0].N);
  const bool ok2 = usable(o.idx[1], h.lv[1].N);
  const bool ok3 = usable(o.idx[2], h.lv[2].N);
  const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
  if (ok1 && ok2 && ok3 && sph_r2(dx, dy, dz, h.lv[0].inv_q) < h.lv[0].R2) o.cls = SBX_CORE;
  else if (ok2 && ok3 && sph_r2(dx, dy, dz, h.lv[1].inv_q) < h.lv[1].R2) o.cls = SBX_RING;
  else if (ok3) o.cls = SBX_OUTER;
  else o.cls = SBX_LOST;
}

// Outside the usable cells of the fixed global grid (the outer level of
// galaxy 0, shared by all galaxies, or the single grid).
__device__ __forceinline__ bool outside_global(const SysDev& sys, double x, double y, double z) {
  const HierDev& h = sys.h[0];
  int i[3];
  if (h.n_levels == 1) {
    cell3(h.lv[0], h.centre, x, y, z, i);
    return !usable(i, h.lv[0].N);
  }
  cell3(h.lv[2], h.outer_c, x, y, z, i);
  return !usable(i, h.lv[2].N);
}

// ------------------------------------------------------------ reductions --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum vals[0..nv) over the block (256 threads) in a fixed order; thread k
// writes total k to out[k * stride].
// Only the first nv (<= NV) values are reduced; the rest are written as 0.
template <int NV>
__device__ __forceinline__ void block_sum_store(const double* vals, double* out, int nv = NV,
                                                int stride = 1) {
  __shared__ double red[4][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < nv) {
      const double s = wave_sum(vals[k]);
      if (lane == 0) red[wave][k] = s;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += blockDim.x)
    out[(size_t)k * stride] = k < nv ? ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k] : 0.0;
}



// Cross-lane moves by DPP (data-parallel primitives of the VALU, no LDS
// round trip).  Lanes whose source is outside the pattern, or whose row is
// masked off, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_t(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_u32<CTRL, ROWS>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = dpp_u32<CTRL, ROWS>((uint32_t)u);
    const uint32_t hi = dpp_u32<CTRL, ROWS>((uint32_t)(u >> 32));
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}
constexpr int kDppRowShr = 0x110;    // + n: from lane - n of the same row of 16
constexpr int kDppBcast15 = 0x142;   // lane 15 of each row to the next row
constexpr int kDppBcast31 = 0x143;   // lane 31 to rows 2 and 3
constexpr int kDppWaveShr1 = 0x138;  // from lane - 1
constexpr int kDppWaveShl1 = 0x130;  // from lane + 1

// One step of a segmented inclusive scan: add the partial from the source
// lane unless a segment starts at or before this lane within the span.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ void seg_step(T& s, uint32_t& f) {
  const T su = dpp_t<CTRL, ROWS>(s);
  const uint32_t fu = dpp_u32<CTRL, ROWS>(f);
  if (!f) s += su;
  f |= fu;
}

// Segmented sum over runs of equal keys in consecutive lanes: returns, in the
// last lane of each run (tail = true), the run's total.  All 64 lanes call it.
// Scan within rows of 16 lanes (shifts 1, 2, 4, 8), then across rows by the
// row broadcasts of lanes 15 and 31.
template <typename T>
__device__ __forceinline__ T wave_run_sum(uint32_t key, T val, bool& tail) {
  const int lane = threadIdx.x & 63;
  const uint32_t kprev = dpp_u32<kDppWaveShr1, 0xf>(key);
  const uint32_t knext = dpp_u32<kDppWaveShl1, 0xf>(key);
  uint32_t f = (lane == 0) || (kprev != key);
  T s = val;
  seg_step<kDppRowShr + 1, 0xf>(s, f);
  seg_step<kDppRowShr + 2, 0xf>(s, f);
  seg_step<kDppRowShr + 4, 0xf>(s, f);
  seg_step<kDppRowShr + 8, 0xf>(s, f);
  seg_step<kDppBcast15, 0xa>(s, f);
  seg_step<kDppBcast31, 0xc>(s, f);
  tail = (lane == 63) || (knext != key);
  return s;
}

// Sum over the 64 lanes by a DPP scan; the total is valid in lane 63 only.
template <typename T>
__device__ __forceinline__ T wave_total63(T v) {
  v += dpp_t<kDppRowShr + 1, 0xf>(v);
  v += dpp_t<kDppRowShr + 2, 0xf>(v);
  v += dpp_t<kDppRowShr + 4, 0xf>(v);
  v += dpp_t<kDppRowShr + 8, 0xf>(v);
  v += dpp_t<kDppBcast15, 0xa>(v);
  v += dpp_t<kDppBcast31, 0xc>(v);
  return v;
}

// Key of a deposit target: grid slot (galaxy * 5 + slot) in the top bits,
// cell index in the low 24 bits (N <= 256).
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t dep_key(int g, int slot, const LevelDev& L, const int* i) {
  return ((uint32_t)(g * kSlots + slot) << 24) |
         (uint32_t)(((i[2] * L.N) + i[1]) * L.N + i[0]);
}


// ------------------------------------------------------------------ Eq. 8 --
// Acceleration (+grad Phi) and Phi at the particle from one field on one
// level: central differences plus the second-order Taylor terms, the offset
// Delta = (x - c) - (i - N/2) * l measured from the cell centre.
// Three consecutive values of a grid row (x-1, x, x+1): one 12-byte load in
// FP32, a 16-byte and an 8-byte load in FP64.
template <typename T>
struct Row3 {
  T m, c, p;
};
typedef float f32x3 __attribute__((ext_vector_type(3), aligned(4)));
typedef double f64x2 __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ Row3<float> row3(gp<const float> q) {
  const f32x3 v = *(gp<const f32x3>)(q - 1);
  return {v.x, v.y, v.z};
}
__device__ __forceinline__ Row3<double> row3(gp<const double> q) {
  const f64x2 v = *(gp<const f64x2>)(q - 1);
  return {v.x, v.y, q[1]};
}

template <bool TAYLOR, typename T>
__device__ __forceinline__ void eq8(const T* __restrict__ F, const LevelDev& L, const int* id,
                                    double dx, double dy, double dz, T* a, T& phi, bool want_phi) {
  const ptrdiff_t sy = L.N, sz = (ptrdiff_t)L.N * L.N;
  const gp<const T> P = glb(F) + ((ptrdiff_t)id[2] * sz + (ptrdiff_t)id[1] * sy + id[0]);
  const T Dx = (T)(dx - ((double)id[0] - L.half) * L.l);
  const T Dy = (T)(dy - ((double)id[1] - L.half) * L.l);
  const T Dz = (T)(dz - ((double)id[2] - L.half) * L.lz);
  const T i2l = (T)L.c_2l, i2lz = (T)L.c_2lz;
  // the 19-point stencil as 5 rows of three along x and 4 single values
  const Row3<T> r00 = row3(P), rp0 = row3(P + sy), rm0 = row3(P - sy);
  const Row3<T> r0p = row3(P + sz), r0m = row3(P - sz);
  // the yz diagonals are loaded with the rows (one round trip per field;
  // every stencil point lies inside the grid for any usable cell)
  const T dpp = P[sy + sz], dmp = P[-sy + sz], dmm = P[-sy - sz], dpm = P[sy - sz];
  const T p0 = r00.c, xp = r00.p, xm = r00.m;
  const T yp = rp0.c, ym = rm0.c, zp = r0p.c, zm = r0m.c;
  const T gx = (xp - xm) * i2l, gy = (yp - ym) * i2l, gz = (zp - zm) * i2lz;
  if constexpr (!TAYLOR) {
    a[0] += gx;
    a[1] += gy;
    a[2] += gz;
    if (want_phi) phi += p0 + gx * Dx + gy * Dy + gz * Dz;
    return;
  }
  const T il2 = (T)L.c_l2, ilz2 = (T)L.c_lz2;
  const T i4xy = (T)L.c_4ll, i4xz = (T)L.c_4llz;
  const T hxx = (xp + xm - (T)2 * p0) * il2;
  const T hyy = (yp + ym - (T)2 * p0) * il2;
  const T hzz = (zp + zm - (T)2 * p0) * ilz2;
  const T hxy = (rp0.p - rp0.m + rm0.m - rm0.p) * i4xy;
  const T hxz = (r0p.p - r0p.m + r0m.m - r0m.p) * i4xz;
  const T hyz = (dpp - dmp + dmm - dpm) * i4xz;
  a[0] += gx + hxx * Dx + hxy * Dy + hxz * Dz;
  a[1] += gy + hyy * Dy + hxy * Dx + hyz * Dz;
  a[2] += gz + hzz * Dz + hxz * Dx + hyz * Dy;
  if (want_phi)
    phi += p0 + gx * Dx + gy * Dy + gz * Dz +
           (T)0.5 * (hxx * Dx * Dx + hyy * Dy * Dy + hzz * Dz * Dz) + hxy * Dx * Dy +
           hxz * Dx * Dz + hyz * Dy * Dz;
  // one field's stencil in registers at a time: letting the scheduler
  // gather the next field's ahead of this arithmetic took more registers
  // and measured slower
  __builtin_amdgcn_sched_barrier(0);
}

// Sum over galaxies of the fields the grid-selection rule gives each class:
// core -> grid 1 + grid 3 + grid 5, ring -> (2 + 3) + grid 5, outer -> (4 + 5).
// With merge5 every class's grid 5 term is the shared summed grid 5, read
// once per particle (Sec. 2.1: each class's sum contains grid 5).
template <bool TAYLOR, typename T>
__device__ __forceinline__ void particle_field(const SysDev& sys, const double* centres,
                                               const GridsDev<T>& F, double x, double y,
                                               double z, T* a, T& phi, bool want_phi) {
  const bool m5 = sys.merge5 != 0;
  bool live5 = false;
  int i5[3] = {0, 0, 0};
  for (int g = 0; g < sys.ngal; ++g) {
    const HierDev& h = sys.h[g];
    const double* c = centres + 3 * g;
    Classified cl;
    classify(h, c, x, y, z, cl);
    const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
    if (h.n_levels == 1) {
      if (cl.cls == SBX_OUTER) eq8<TAYLOR>(F.g[g][0], h.lv[0], cl.idx[0], dx, dy, dz, a, phi, want_phi);
      continue;
    }
    const double ox = x - h.outer_c[0], oy = y - h.outer_c[1], oz = z - h.outer_c[2];
    switch (cl.cls) {
      case SBX_CORE:
        eq8<TAYLOR>(F.g[g][0], h.lv[0], cl.idx[0], dx, dy, dz, a, phi, want_phi);
        eq8<TAYLOR>(F.g[g][1], h.lv[1], cl.idx[1], dx, dy, dz, a, phi, want_phi);
        if (!m5) eq8<TAYLOR>(F.g[g][3], h.lv[2], cl.idx[2], ox, oy, oz, a, phi, want_phi);
        break;
      case SBX_RING:
        eq8<TAYLOR>(F.g[g][2], h.lv[1], cl.idx[1], dx, dy, dz, a, phi, want_phi);
        if (!m5) eq8<TAYLOR>(F.g[g][3], h.lv[2], cl.idx[2], ox, oy, oz, a, phi, want_phi);
        break;
      case SBX_OUTER:
        eq8<TAYLOR>(F.g[g][4], h.lv[2], cl.idx[2], ox, oy, oz, a, phi, want_phi);
        break;
      default:
        break;
    }
    if (m5 && g == 0 && cl.cls != SBX_LOST) {
      live5 = true;
      i5[0] = cl.idx[2][0];
      i5[1] = cl.idx[2][1];
      i5[2] = cl.idx[2][2];
    }
  }
  if (live5) {
    const HierDev& h = sys.h[0];
    eq8<TAYLOR>(F.g[0][3], h.lv[2], i5, x - h.outer_c[0], y - h.outer_c[1], z - h.outer_c[2], a, phi,
               want_phi);
  }
}


// Rows of the force pass partials (mirrors force_blocks on the host).
__device__ __forceinline__ int force_blocks_dev(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > kForceBlocksMax ? kForceBlocksMax : b));
}


// Zero n elements at g (a device allocation, 16-byte aligned) with block lb
// of nb (256 threads each): 16-byte global stores, then the tail.
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ void zero_block(T* g, size_t n, int lb, int nb) {
  constexpr size_t per = 16 / sizeof(T);
  const size_t n16 = n / per;
  const gp<u32x4> G = glb((u32x4*)g);
  for (size_t k = (size_t)lb * 256 + threadIdx.x; k < n16; k += (size_t)nb * 256) G[k] = u32x4{0u, 0u, 0u, 0u};
  if (lb == 0 && threadIdx.x < n - n16 * per) glb(g)[n16 * per + threadIdx.x] = (T)0;
}

// ------------------------------------------------------------- instances --
__device__ __forceinline__ int span_inst(const Span& sp, int b) {
  int i = 0;
  while (i + 1 < sp.ninst && sp.start[i + 1] <= b) ++i;
  return i;
}

// Copy a trivially copyable record into LDS with the whole block.
template <typename R>
__device__ __forceinline__ void stage(R* dst, const R* src) {
  static_assert(sizeof(R) % 4 == 0, "word copy");
  const uint32_t* s = (const uint32_t*)src;
  uint32_t* d = (uint32_t*)dst;
  for (int k = threadIdx.x; k < (int)(sizeof(R) / 4); k += blockDim.x) d[k] = s[k];
}

static Span make_span(const std::vector<InstInfo>& info, int64_t (*blocks)(const InstInfo&)) {
  Span sp;
  sp.ninst = (int)info.size();
  sp.start[0] = 0;
  for (int i = 0; i < sp.ninst; ++i) sp.start[i + 1] = sp.start[i] + (int)blocks(info[i]);
  return sp;
}

int force_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > kForceBlocksMax ? kForceBlocksMax : b));
}

static int64_t blocks_particles(const InstInfo& f) { return f.n > 0 ? (f.n + 255) / 256 : 1; }
static int64_t blocks_force(const InstInfo& f) { return force_blocks(f.n); }
static int64_t blocks_deposit(const InstInfo& f) { return f.n > 0 ? (f.n + kDepChunk - 1) / kDepChunk : 1; }
static int64_t blocks_red(const InstInfo&) { return kRedBlocks; }
static int64_t blocks_dm(const InstInfo& f) {
  const int64_t b = (int64_t)((f.dm_elems + 1023) / 1024);
  return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}
static int64_t blocks_sort(const InstInfo& f) { return f.n > 0 ? (f.n + 255) / 256 : 1; }
static int64_t blocks_grid(const InstInfo& f) {
  const int64_t b = (int64_t)((f.grid_elems + 1023) / 1024);
  return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

// ------------------------------------------------------------ zero grids --
// With the fixed-point assignment the cell masses are not summed in place:
// the conversion pass writes every one of them after the assignment (and
// leaves the accumulators cleared), so there is nothing to clear.
template <typename T>
__global__ void __launch_bounds__(256) k_zero_grids(const InstDev<T>* __restrict__ inst, Span sp) {
  const int i = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[i], nb = sp.start[i + 1] - sp.start[i];
  if (!inst[i].fix) zero_block(inst[i].grid_block, inst[i].grid_elems, lb, nb);
}

// ------------------------------------------------------ loss test and COM --
template <typename T>
__global__ void __launch_bounds__(256)
    k_pre(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii], nb = sp.start[ii + 1] - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  const PartDev<T> p = I.p[cur[ii]];
  const gp<const T> X0 = glb((const T*)p.x[0]), X1 = glb((const T*)p.x[1]), X2 = glb((const T*)p.x[2]);
  const SysDev& sys = I.sys;
  double acc[kPreVals];
#pragma unroll
  for (int k = 0; k < kPreVals; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)nb * blockDim.x;
  for (int64_t i = (int64_t)lb * blockDim.x + threadIdx.x; i < p.n; i += stride) {
    if (p.lost[i]) continue;
    const double x = (double)X0[i], y = (double)X1[i], z = (double)X2[i];
    if (outside_global(sys, x, y, z)) {
      p.lost[i] = 1;
      continue;
    }
    const int g = p.gal[i];
#pragma unroll
    for (int gg = 0; gg < kMaxGal; ++gg) {
      if (gg == g && sys.h[gg].centring == SBX_CENTRE_COM) {
        const double m = (double)p.m[i];
        acc[4 * gg + 0] += m;
        acc[4 * gg + 1] += m * x;
        acc[4 * gg + 2] += m * y;
        acc[4 * gg + 3] += m * z;
      }
    }
  }
  block_sum_store<kPreVals>(acc, I.pre_partial + lb, 4 * sys.ngal, kRedBlocks);
}

// Sum of rows values (fixed order) into out[0]; one block of 256 threads.
__global__ void __launch_bounds__(256) k_reduce_one(const double* __restrict__ part, int rows,
                                                    double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) s += part[r];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// One block per instance: column sums of the partial rows, then the
// centres.  The partials are stored column by column (value v of block row
// r at v * rows_max + r), so each column is one contiguous run: per galaxy
// the threads load eight rows of its four columns per round (32 loads in
// flight; one block is all the kernel has, so it is bound by these round
// trips), then the block reduces each column in a fixed order (wavefront
// butterfly, then the four waves in order).  Galaxies
// centred on their density maximum take their sums from dm_partial when
// `density` is set and keep their current centre otherwise.
template <typename T>
__device__ __forceinline__ void centres_of(const InstDev<T>& I, int from_com, int density) {
  __shared__ double red[4][kPreVals];
  __shared__ double sums[kPreVals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool dm_on = density && I.dm_partial;
  for (int g = 0; g < I.sys.ngal; ++g) {
    const bool dm = I.sys.h[g].centring == SBX_CENTRE_DENSITY;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (!dm || dm_on) {
      const bool com = from_com && !dm;
      const size_t cs = com ? kForceBlocksMax : kRedBlocks;  // column stride
      const gp<const double> col = glb((const double*)(dm ? I.dm_partial : (com ? I.com_partial : I.pre_partial)) + 4 * g * cs);
      const int rows = com ? force_blocks_dev(I.n) : kRedBlocks;
      // the galaxy's four columns, eight rows each per round, loads together
      for (int r0 = threadIdx.x; r0 < rows; r0 += 8 * 256) {
        double x[4][8];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int r = r0 + u * 256;
            x[k][u] = r < rows ? col[k * cs + r] : 0.0;
          }
#pragma unroll
        for (int k = 0; k < 4; ++k)
          a[k] += ((x[k][0] + x[k][1]) + (x[k][2] + x[k][3])) + ((x[k][4] + x[k][5]) + (x[k][6] + x[k][7]));
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double w = wave_sum(a[k]);
      if (lane == 0) red[wave][4 * g + k] = w;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 4 * I.sys.ngal) {
    const int v = threadIdx.x;
    sums[v] = ((red[0][v] + red[1][v]) + red[2][v]) + red[3][v];
  }
  __syncthreads();
  if ((int)threadIdx.x < I.sys.ngal) {
    const int g = threadIdx.x;
    const HierDev& h = I.sys.h[g];
    double c[3] = {h.centre[0], h.centre[1], h.centre[2]};
    const bool dm = h.centring == SBX_CENTRE_DENSITY;
    if (dm) {
      c[0] = I.centres[3 * g + 0];
      c[1] = I.centres[3 * g + 1];
      c[2] = I.centres[3 * g + 2];
    }
    if ((h.centring == SBX_CENTRE_COM || (dm && dm_on)) && sums[4 * g] > 0.0) {
      c[0] = sums[4 * g + 1] / sums[4 * g];
      c[1] = sums[4 * g + 2] / sums[4 * g];
      c[2] = sums[4 * g + 3] / sums[4 * g];
    }
    I.centres[3 * g + 0] = c[0];
    I.centres[3 * g + 1] = c[1];
    I.centres[3 * g + 2] = c[2];
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_centres(const InstDev<T>* __restrict__ inst, int from_com, int density) {
  centres_of(inst[blockIdx.x], from_com, density);
}

// The grid clearing of the next deposit and, in each instance's first
// block, the centres from the sums the last moving force pass left (one
// launch instead of two when no density centring needs the particles).
template <typename T>
__global__ void __launch_bounds__(256)
    k_zero_centres(const InstDev<T>* __restrict__ inst, Span sp) {
  const int i = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[i], nb = sp.start[i + 1] - sp.start[i];
  if (lb == 0) centres_of(inst[i], 1, 0);
  if (!inst[i].fix) zero_block(inst[i].grid_block, inst[i].grid_elems, lb, nb);
}

// ------------------------------------------------ density-maximum centring --
// Reading of Sec. 2.1 (the inner and middle grids follow the density maximum
// of their galaxy): the galaxy's live particle masses are binned on the N^3
// cells (Eq. 7) of its inner grid placed at the current centre, each as the
// integer floor(m 2^s), s = 62 - e - b (the largest mass of the instance is
// below 2^e, b is the bit length of n), so every cell total fits in 62 bits
// and does not depend on the order of the atomic adds.  The densest cell
// (ties: lowest (z, y, x) index) and the FP64 mass centre of the live
// particles in its 3x3x3 block give the new centre.

__device__ __forceinline__ int dm_shift(unsigned long long mmax_bits, int64_t n) {
  int e = 0;
  (void)frexp(__longlong_as_double((long long)mmax_bits), &e);
  const int b = n > 0 ? 64 - __clzll((long long)n) : 0;
  return 62 - e - b;
}

// Zero the histogram.
template <typename T>
__global__ void __launch_bounds__(256) k_dm_zero(const InstDev<T>* __restrict__ inst, Span sp) {
  const int i = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[i], nb = sp.start[i + 1] - sp.start[i];
  const InstDev<T>& I = inst[i];
  if (!I.dm_hist) return;
  for (size_t k = (size_t)lb * 256 + threadIdx.x; k < I.dm_elems; k += (size_t)nb * 256) I.dm_hist[k] = 0ull;
}

// Largest particle mass (taken when the particles are loaded; the masses do
// not change afterwards): the bit patterns of non-negative doubles order like
// the values.  *out must be zero on entry.
template <typename T>
__global__ void __launch_bounds__(256) k_mass_max(const T* __restrict__ m, int64_t n,
                                                  unsigned long long* __restrict__ out) {
  const gp<const T> M = glb(m);
  unsigned long long mx = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    mx = max(mx, (unsigned long long)__double_as_longlong((double)M[i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (unsigned long long)__shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0 && mx) atomicMax(out, mx);
}

// Integer cell masses of every density-centred galaxy's live particles (one
// particle per thread).
template <typename T>
__global__ void __launch_bounds__(256)
    k_dm_hist(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  __shared__ SysDev sys;
  __shared__ double cen[3 * kMaxGal];
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  if (!I.dm_hist) return;
  const PartDev<T> p = I.p[cur[ii]];
  stage(&sys, &I.sys);
  if (threadIdx.x < 3 * kMaxGal) cen[threadIdx.x] = I.centres[threadIdx.x];
  __syncthreads();
  const int shift = dm_shift(*I.dm_mmax, I.n);
  const int N = sys.h[0].lv[0].N;
  const uint32_t N3 = (uint32_t)N * N * N;
  const int64_t i = (int64_t)lb * 256 + threadIdx.x;
  uint32_t key = kNoKey;  // lanes past the end take part in the wave sum
  unsigned long long q = 0ull;
  if (i < p.n && !glb((const uint8_t*)p.lost)[i]) {
    const int g = glb((const int8_t*)p.gal)[i];
    const HierDev& h = sys.h[g];
    if (h.centring == SBX_CENTRE_DENSITY) {
      int c[3];
      cell3(h.lv[0], cen + 3 * g, (double)glb((const T*)p.x[0])[i], (double)glb((const T*)p.x[1])[i],
            (double)glb((const T*)p.x[2])[i], c);
      if (c[0] >= 0 && c[0] < N && c[1] >= 0 && c[1] < N && c[2] >= 0 && c[2] < N) {
        key = (uint32_t)g * N3 + ((uint32_t)c[2] * N + c[1]) * N + c[0];
        q = (unsigned long long)floor(ldexp((double)glb((const T*)p.m)[i], shift));
      }
    }
  }
  bool tail;
  const unsigned long long s = wave_run_sum<unsigned long long>(key, q, tail);
  if (tail && key != kNoKey) atomic_add_g(glb(I.dm_hist + key), s);
}

// Larger total wins; equal totals go to the lower index.
__device__ __forceinline__ void dm_better(unsigned long long& v, unsigned long long& k,
                                          unsigned long long v2, unsigned long long k2) {
  if (v2 > v || (v2 == v && k2 < k)) {
    v = v2;
    k = k2;
  }
}

__device__ __forceinline__ void dm_block_best(unsigned long long& v, unsigned long long& k) {
  __shared__ unsigned long long sv[256], sk[256];
  sv[threadIdx.x] = v;
  sk[threadIdx.x] = k;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      unsigned long long a = sv[threadIdx.x], b = sk[threadIdx.x];
      dm_better(a, b, sv[threadIdx.x + w], sk[threadIdx.x + w]);
      sv[threadIdx.x] = a;
      sk[threadIdx.x] = b;
    }
    __syncthreads();
  }
  v = sv[0];
  k = sk[0];
}

// Densest cell, first stage: grid (kArgParts, kMaxGal, instances).
template <typename T>
__global__ void __launch_bounds__(256) k_dm_arg1(const InstDev<T>* __restrict__ inst) {
  const InstDev<T>& I = inst[blockIdx.z];
  const int g = blockIdx.y;
  if (!I.dm_hist || g >= I.sys.ngal || I.sys.h[g].centring != SBX_CENTRE_DENSITY) return;
  const int N = I.sys.h[0].lv[0].N;
  const size_t N3 = (size_t)N * N * N;
  const unsigned long long* hg = I.dm_hist + (size_t)g * N3;
  unsigned long long v = 0ull, k = ~0ull;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N3; c += (size_t)kArgParts * 256)
    dm_better(v, k, hg[c], c);
  dm_block_best(v, k);
  if (threadIdx.x == 0) {
    unsigned long long* part = I.dm_aux + kMaxGal + 2 * ((size_t)g * kArgParts + blockIdx.x);
    part[0] = v;
    part[1] = k;
  }
}

// Second stage: grid (kMaxGal, instances); the cell, or all ones when the
// galaxy has no mass on its inner grid.
template <typename T>
__global__ void __launch_bounds__(256) k_dm_arg2(const InstDev<T>* __restrict__ inst) {
  const InstDev<T>& I = inst[blockIdx.y];
  const int g = blockIdx.x;
  if (!I.dm_hist || g >= I.sys.ngal || I.sys.h[g].centring != SBX_CENTRE_DENSITY) return;
  const unsigned long long* part = I.dm_aux + kMaxGal + 2 * (size_t)g * kArgParts;
  unsigned long long v = 0ull, k = ~0ull;
  for (int r = threadIdx.x; r < kArgParts; r += 256) dm_better(v, k, part[2 * r], part[2 * r + 1]);
  dm_block_best(v, k);
  if (threadIdx.x == 0) I.dm_aux[g] = v > 0ull ? k : ~0ull;
}

// Mass sums of each density-centred galaxy's live particles in the 3x3x3
// block around its densest cell (rows of dm_partial).
template <typename T>
__global__ void __launch_bounds__(256)
    k_dm_window(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  __shared__ SysDev sys;
  __shared__ double cen[3 * kMaxGal];
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii], nb = sp.start[ii + 1] - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  if (!I.dm_hist) return;
  const PartDev<T> p = I.p[cur[ii]];
  stage(&sys, &I.sys);
  if (threadIdx.x < 3 * kMaxGal) cen[threadIdx.x] = I.centres[threadIdx.x];
  __syncthreads();
  const gp<const T> X0 = glb((const T*)p.x[0]), X1 = glb((const T*)p.x[1]), X2 = glb((const T*)p.x[2]);
  const gp<const T> M = glb((const T*)p.m);
  const gp<const uint8_t> LOST = glb((const uint8_t*)p.lost);
  const gp<const int8_t> GAL = glb((const int8_t*)p.gal);
  const int N = sys.h[0].lv[0].N;
  int best[kMaxGal][3];
#pragma unroll
  for (int g = 0; g < kMaxGal; ++g) {
    const unsigned long long k = g < sys.ngal && sys.h[g].centring == SBX_CENTRE_DENSITY
                                     ? I.dm_aux[g] : ~0ull;
    if (k == ~0ull) {
      best[g][0] = best[g][1] = best[g][2] = -1000;  // never within one cell
    } else {
      best[g][0] = (int)(k % N);
      best[g][1] = (int)((k / N) % N);
      best[g][2] = (int)(k / ((unsigned long long)N * N));
    }
  }
  double acc[kPreVals];
#pragma unroll
  for (int k = 0; k < kPreVals; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)lb * 256 + threadIdx.x; i < p.n; i += (int64_t)nb * 256) {
    if (LOST[i]) continue;
    const int g = GAL[i];
    const HierDev& h = sys.h[g];
    if (h.centring != SBX_CENTRE_DENSITY) continue;
    const double x = (double)X0[i], y = (double)X1[i], z = (double)X2[i];
    int c[3];
    cell3(h.lv[0], cen + 3 * g, x, y, z, c);
#pragma unroll
    for (int gg = 0; gg < kMaxGal; ++gg) {
      if (gg == g && abs(c[0] - best[gg][0]) <= 1 && abs(c[1] - best[gg][1]) <= 1 &&
          abs(c[2] - best[gg][2]) <= 1) {
        const double m = (double)M[i];
        acc[4 * gg + 0] += m;
        acc[4 * gg + 1] += m * x;
        acc[4 * gg + 2] += m * y;
        acc[4 * gg + 3] += m * z;
      }
    }
  }
  block_sum_store<kPreVals>(acc, I.dm_partial + lb, 4 * sys.ngal, kRedBlocks);
}

// ---------------------------------------------------------- mass deposit --
// Mass assignment on cell-sorted particles.  Each block takes a contiguous
// chunk of particles.  The deposits on a particle's finest level (the level
// the sort orders by) are combined across lanes of a wavefront that hit the
// same cell (segmented wave sum) and added to global memory straight from the
// run tails: consecutive runs hit neighbouring cells, so these atomics are
// close to coalesced.  Deposits on coarser levels repeat across many
// particles of a chunk; they are summed in the wavefront, accumulated in an
// LDS hash table of the block's coarse cells and flushed with one global
// atomic per distinct cell (targets that find no free entry within a few
// probes go straight to global memory).
//
// Sources of the five grids (Sec. 2.1): core -> grid 1, grid 2, grid 4;
// ring -> grid 3, grid 4; outer -> grid 5.  The potentials of grids 2 and 4
// are only used summed with those of grids 3 and 5, and the solve is linear,
// so only the sums 2+3 and 4+5 are solved; every mass is assigned once, to
// its own grid, and the solves of the summed grids add their two sources as
// they read them (see the slot layout in particles.h).
constexpr int kDepTableBits = 11;
constexpr int kDepTable = 1 << kDepTableBits;  // LDS hash entries
constexpr int kDepProbes = 8;

template <typename T>
__device__ __forceinline__ T* slot_ptr(const GridsDev<T>& G, uint32_t key) {
  const int gs = (int)(key >> 24);
  const int g = gs / kSlots, slot = gs - g * kSlots;
  return G.g[g][slot] + (key & 0xFFFFFFu);
}

//
// FIX: the fixed-point form.  Every mass enters as the integer
// floor(m 2^s), s = 62 - e - b (the largest mass of the instance is below
// 2^e, b is the bit length of its particle count; the scale of the
// density-maximum centring), so every cell total fits in 62 bits; the sums
// are exact 64-bit integer sums in any order, into the accumulators I.fix
// (one per mass-grid element), and k_fix_convert turns them into cell
// masses.  Cell masses then do not depend on the order of the adds.
template <typename T, bool FIX>
__global__ void __launch_bounds__(256)
    k_deposit(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  using V = std::conditional_t<FIX, unsigned long long, T>;
  __shared__ uint32_t tkey[kDepTable];
  __shared__ V tval[kDepTable];
  // per-galaxy data staged in LDS: lanes index it by their own galaxy
  __shared__ SysDev sys;
  __shared__ GridsDev<T> G;
  __shared__ double cen[3 * kMaxGal];
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  const PartDev<T> p = I.p[cur[ii]];
  const gp<const T> X0 = glb((const T*)p.x[0]), X1 = glb((const T*)p.x[1]), X2 = glb((const T*)p.x[2]);
  const gp<const T> Mv = glb((const T*)p.m);
  const gp<const uint8_t> LOST = glb((const uint8_t*)p.lost);
  const gp<const int8_t> GAL = glb((const int8_t*)p.gal);
  stage(&sys, &I.sys);
  stage(&G, &I.G);
  if (threadIdx.x < 3 * kMaxGal) cen[threadIdx.x] = I.centres[threadIdx.x];
  for (int k = threadIdx.x; k < kDepTable; k += 256) {
    tkey[k] = kNoKey;
    tval[k] = (V)0;
  }
  int shift = 0;
  if constexpr (FIX) shift = dm_shift(*I.dm_mmax, I.n);
  // the accumulator of a deposit key: the mass grid element itself, or its
  // fixed-point accumulator at the same offset in the grid block
  auto target = [&](uint32_t key) -> gp<V> {
    T* cell = slot_ptr(G, key);
    if constexpr (FIX) return glb(I.fix + (cell - I.grid_block));
    else return glb(cell);
  };
  __syncthreads();
  const int64_t base = (int64_t)lb * kDepChunk;
  // The next particle is loaded one iteration ahead, every field whatever
  // its flag, so that the loads go out together and the flag is waited for
  // only where it is used (l = 1 marks no particle).
  auto fetch = [&](int64_t q, uint8_t& l, int& g, T& x, T& y, T& z, T& mm) {
    l = 1;
    if (q < p.n) {
      l = LOST[q];
      g = GAL[q];
      x = X0[q];
      y = X1[q];
      z = X2[q];
      mm = Mv[q];
    }
  };
  uint8_t lnx = 1;
  int gn = 0;
  T xn = (T)0, yn = (T)0, zn = (T)0, mn = (T)0;
  fetch(base + threadIdx.x, lnx, gn, xn, yn, zn, mn);
  for (int j = 0; j < kDepChunk / 256; ++j) {
    const bool ok = lnx == 0;
    const int g = gn;
    const T xs = xn, ys = yn, zs = zn, ms = mn;
    if (j + 1 < kDepChunk / 256) fetch(base + (j + 1) * 256 + threadIdx.x, lnx, gn, xn, yn, zn, mn);
    // fine: key on the finest level, or kNoKey; coarse keys c1, c2 go
    // through the table
    uint32_t fine = kNoKey, c1 = kNoKey, c2 = kNoKey;
    V m = (V)0;
    if (ok) {
      const HierDev& h = sys.h[g];
      const double x = (double)xs, y = (double)ys, z = (double)zs;
      Classified c;
      classify(h, cen + 3 * g, x, y, z, c);
      if constexpr (FIX) m = (V)ldexp((double)ms, shift);  // floor: non-negative, truncated
      else m = ms;
      if (h.n_levels == 1) {
        if (c.cls == SBX_OUTER) fine = dep_key(g, 0, h.lv[0], c.idx[0]);
      } else if (c.cls == SBX_CORE) {
        fine = dep_key(g, 0, h.lv[0], c.idx[0]);        // grid 1
        c1 = dep_key(g, kSlotG2, h.lv[1], c.idx[1]);    // grid 2
        c2 = dep_key(g, kSlotG4, h.lv[2], c.idx[2]);    // grid 4
      } else if (c.cls == SBX_RING) {
        fine = dep_key(g, 1, h.lv[1], c.idx[1]);        // grid 3
        c2 = dep_key(g, kSlotG4, h.lv[2], c.idx[2]);    // grid 4
      } else if (c.cls == SBX_OUTER) {
        fine = dep_key(sys.merge5 ? 0 : g, 3, h.lv[2], c.idx[2]);  // grid 5 (summed if merged)
      }
    }
    {
      bool tail;
      const V s = wave_run_sum<V>(fine, m, tail);
      if (tail && fine != kNoKey) atomic_add_g(target(fine), s);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const uint32_t key = r == 0 ? c1 : c2;
      bool tail;
      V s;
      // a coarse cell is usually the same for the whole wavefront: then a
      // plain wavefront sum (in lane 63) replaces the segmented one
      const uint32_t k0 = __builtin_amdgcn_readfirstlane(key);
      if (__ballot(key != k0) == 0ull) {
        s = wave_total63<V>(m);
        tail = (threadIdx.x & 63) == 63;
      } else {
        s = wave_run_sum<V>(key, m, tail);
      }
      if (tail && key != kNoKey) {
        uint32_t hslot = (key * 2654435761u) >> (32 - kDepTableBits);
        bool done = false;
        for (int q = 0; q < kDepProbes && !done; ++q) {
          const uint32_t old = atomicCAS(tkey + hslot, kNoKey, key);
          if (old == kNoKey || old == key) {
            atomicAdd(tval + hslot, s);
            done = true;
          } else {
            hslot = (hslot + 1) & (kDepTable - 1);
          }
        }
        if (!done) atomic_add_g(target(key), s);
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kDepTable; k += 256) {
    const uint32_t key = tkey[k];
    if (key != kNoKey) atomic_add_g(target(key), tval[k]);
  }
}

// Fixed-point mass assignment, second step: every accumulator of the
// instance's mass grids becomes its cell mass (T)(sum 2^-s) (the integer
// converted to float64 with one rounding, then scaled exactly) and is
// cleared for the next assignment.
template <typename T>
__global__ void __launch_bounds__(256) k_fix_convert(const InstDev<T>* __restrict__ inst, Span sp) {
  const int i = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[i], nb = sp.start[i + 1] - sp.start[i];
  const InstDev<T>& I = inst[i];
  const int shift = dm_shift(*I.dm_mmax, I.n);
  const gp<unsigned long long> F = glb(I.fix);
  const gp<T> M = glb(I.grid_block);
  for (size_t k = (size_t)lb * 256 + threadIdx.x; k < I.grid_elems; k += (size_t)nb * 256) {
    const unsigned long long q = F[k];
    // both halves exact in float64; their sum rounded once
    const double d = (double)(uint32_t)(q >> 32) * 4294967296.0 + (double)(uint32_t)q;
    M[k] = (T)ldexp(d, -shift);
    F[k] = 0ull;
  }
}

// ----------------------------------------------------------- force + move --
// MODE bits: 1 move, 2 write acc/pot, 4 diagnostics.  The block walks the
// instance's particles in block-uniform strides so that every lane of a
// wavefront takes part in the per-component diagnostic sums.
template <typename T, int MODE>
__global__ void __launch_bounds__(256)
    k_force(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  constexpr bool MOVE = MODE & 1, OUT = MODE & 2, DIAG = MODE & 4;
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii], nb = sp.start[ii + 1] - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  const PartDev<T> p = I.p[cur[ii]];
  const gp<T> X0 = glb(p.x[0]), X1 = glb(p.x[1]), X2 = glb(p.x[2]);
  const gp<T> V0 = glb(p.v[0]), V1 = glb(p.v[1]), V2 = glb(p.v[2]);
  const gp<const T> Mv = glb((const T*)p.m);
  const gp<uint8_t> LOST = glb(p.lost);
  const gp<const int8_t> GAL = glb((const int8_t*)p.gal), COMP = glb((const int8_t*)p.comp);
  const SysDev& sys = I.sys;
  const GridsDev<T>& F = I.G;
  // the centres are read from LDS: a global load of them inside the loop
  // would wait for every load in flight, the next particle's included
  __shared__ double centres[3 * kMaxGal];
  if (threadIdx.x < 3 * kMaxGal) centres[threadIdx.x] = I.centres[threadIdx.x];
  __syncthreads();
  const T dt = (T)I.dt;
  const double dtd = I.dt;
  // diagnostics: per-component sums per wavefront in LDS (one writer per
  // row, fixed order), disc and lost counts in registers
  __shared__ double wacc[DIAG ? 4 : 1][DIAG ? kDiagDisc : 1];
  double dd[DIAG ? 6 : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if constexpr (DIAG) {
#pragma unroll
    for (int k = 0; k < 6; ++k) dd[k] = 0.0;
    for (int k = threadIdx.x; k < 4 * kDiagDisc; k += 256) (&wacc[0][0])[k] = 0.0;
    __syncthreads();
  }
  // centre-of-mass sums of the moved particles, per wavefront in LDS (one
  // writer per row, fixed order)
  __shared__ double wcom[MOVE ? 4 : 1][MOVE ? kPreVals : 1];
  if constexpr (MOVE) {
    for (int k = threadIdx.x; k < 4 * kPreVals; k += 256) (&wcom[0][0])[k] = 0.0;
    __syncthreads();
  }
  const int64_t stride = (int64_t)nb * blockDim.x;
  // The particle streams are read and written once per pass: their loads
  // and stores are non-temporal, so they do not displace the field rows
  // that neighbouring particles gather from the caches.
  // The next particle's flag and position are loaded one iteration ahead.
  int64_t inext = (int64_t)lb * blockDim.x + threadIdx.x;
  uint8_t lnext = inext < p.n ? __builtin_nontemporal_load(&LOST[inext]) : (uint8_t)1;
  T xn = (T)0, yn = (T)0, zn = (T)0;
  if (inext < p.n) {
    xn = __builtin_nontemporal_load(&X0[inext]);
    yn = __builtin_nontemporal_load(&X1[inext]);
    zn = __builtin_nontemporal_load(&X2[inext]);
  }
  for (int64_t i0 = (int64_t)lb * blockDim.x; i0 < p.n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    const bool valid = i < p.n;
    const bool live = valid && !lnext;
    const T xs = xn, ys = yn, zs = zn;
    inext = i + stride;
    if (inext < p.n) {
      lnext = __builtin_nontemporal_load(&LOST[inext]);
      xn = __builtin_nontemporal_load(&X0[inext]);
      yn = __builtin_nontemporal_load(&X1[inext]);
      zn = __builtin_nontemporal_load(&X2[inext]);
    }
    int dc = -1;                        // component for the diagnostic sums
    double dv[DIAG ? kDiagComp : 1];    // this lane's contribution
    int cg = -1;                        // galaxy for the centre-of-mass sums
    double cm = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    if (valid && !live) {
      if constexpr (OUT) {
        I.acc[3 * i] = I.acc[3 * i + 1] = I.acc[3 * i + 2] = 0.0;
        I.pot[i] = 0.0;
      }
      if constexpr (DIAG) dd[5] += 1.0;
    }
    if (live) {
      const double x = (double)xs, y = (double)ys, z = (double)zs;
      // velocity, galaxy, mass (and component) are loaded before the field
      // gathers, so their memory latency overlaps the gathers'
      T v0 = (T)0, v1 = (T)0, v2 = (T)0, mi = (T)0;
      int gi = 0, ci = 0;
      if constexpr (MOVE || DIAG) {
        v0 = __builtin_nontemporal_load(&V0[i]);
        v1 = __builtin_nontemporal_load(&V1[i]);
        v2 = __builtin_nontemporal_load(&V2[i]);
        gi = __builtin_nontemporal_load(&GAL[i]);
        mi = __builtin_nontemporal_load(&Mv[i]);
      }
      if constexpr (DIAG) ci = COMP[i];
      T a[3] = {(T)0, (T)0, (T)0};
      T phi = (T)0;
      if (sys.taylor)
        particle_field<true>(sys, centres, F, x, y, z, a, phi, OUT || DIAG);
      else
        particle_field<false>(sys, centres, F, x, y, z, a, phi, OUT || DIAG);
      if constexpr (OUT) {
        I.acc[3 * i] = (double)a[0];
        I.acc[3 * i + 1] = (double)a[1];
        I.acc[3 * i + 2] = (double)a[2];
        I.pot[i] = -(double)phi;
      }
      if constexpr (DIAG) {
        const double m = (double)mi;
        const double vx = (double)v0 + 0.5 * dtd * (double)a[0];
        const double vy = (double)v1 + 0.5 * dtd * (double)a[1];
        const double vz = (double)v2 + 0.5 * dtd * (double)a[2];
        dc = ci & (kNComp - 1);
        dv[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
        dv[1] = 0.5 * m * (-(double)phi);
        dv[2] = m * (y * vz - z * vy);
        dv[3] = m * (z * vx - x * vz);
        dv[4] = m * (x * vy - y * vx);
        dv[5] = 1.0;
        if (dc == 0 && gi == 0) {
          const double rx = x - centres[0], ry = y - centres[1];
          const double R = sqrt(rx * rx + ry * ry);
          const double vR = R > 0.0 ? (rx * vx + ry * vy) / R : 0.0;
          dd[0] += vR;
          dd[1] += vR * vR;
          dd[2] += vz;
          dd[3] += vz * vz;
          dd[4] += 1.0;
        }
      }
      if constexpr (MOVE) {
        const T vx = v0 + dt * a[0];
        const T vy = v1 + dt * a[1];
        const T vz = v2 + dt * a[2];
        const T nx = xs + dt * vx, ny = ys + dt * vy, nz = zs + dt * vz;
        __builtin_nontemporal_store(vx, &V0[i]);
        __builtin_nontemporal_store(vy, &V1[i]);
        __builtin_nontemporal_store(vz, &V2[i]);
        __builtin_nontemporal_store(nx, &X0[i]);
        __builtin_nontemporal_store(ny, &X1[i]);
        __builtin_nontemporal_store(nz, &X2[i]);
        const double ex = (double)nx, ey = (double)ny, ez = (double)nz;
        if (outside_global(sys, ex, ey, ez)) {
          LOST[i] = 1;
        } else {
          // centre-of-mass sums of the new positions for the next step
          cg = gi;
          cm = (double)mi;
          cx = cm * ex;
          cy = cm * ey;
          cz = cm * ez;
        }
      }
    }
    if constexpr (MOVE) {
      for (int g = 0; g < sys.ngal; ++g) {
        if (sys.h[g].centring != SBX_CENTRE_COM) continue;
        const bool mine = cg == g;
        const double s0 = wave_total63(mine ? cm : 0.0), s1 = wave_total63(mine ? cx : 0.0);
        const double s2 = wave_total63(mine ? cy : 0.0), s3 = wave_total63(mine ? cz : 0.0);
        if (lane == 63) {
          wcom[wave][4 * g + 0] += s0;
          wcom[wave][4 * g + 1] += s1;
          wcom[wave][4 * g + 2] += s2;
          wcom[wave][4 * g + 3] += s3;
        }
      }
    }
    if constexpr (DIAG) {
      // one pass per component present in the wavefront (uniform loop)
      for (;;) {
        const unsigned long long act = __ballot(dc >= 0);
        if (act == 0ull) break;
        const int c0 = __shfl(dc, __ffsll((long long)act) - 1, 64);
        const bool mine = dc == c0;
#pragma unroll
        for (int k = 0; k < kDiagComp; ++k) {
          const double sum = wave_sum(mine ? dv[k] : 0.0);
          if (lane == 0) wacc[wave][kDiagComp * c0 + k] += sum;
        }
        if (mine) dc = -1;
      }
    }
  }
  if constexpr (DIAG) {
    double* out = I.diag_partial + (size_t)lb * kNDiag;
    block_sum_store<6>(dd, out + kDiagDisc);  // disc sums and lost count (synchronises)
    for (int k = threadIdx.x; k < kDiagDisc; k += 256)
      out[k] = ((wacc[0][k] + wacc[1][k]) + wacc[2][k]) + wacc[3][k];
  }
  if constexpr (MOVE) {
    __syncthreads();
    double* out = I.com_partial + lb;
    for (int k = threadIdx.x; k < 4 * sys.ngal; k += 256)
      out[(size_t)k * kForceBlocksMax] = ((wcom[0][k] + wcom[1][k]) + wcom[2][k]) + wcom[3][k];
  }
}

// One block per (value, instance): column sum of the diagnostics partials.
template <typename T>
__global__ void __launch_bounds__(256) k_diag_final(const InstDev<T>* __restrict__ inst) {
  __shared__ double red[256];
  const InstDev<T>& I = inst[blockIdx.y];
  const int v = blockIdx.x;
  const int rows = force_blocks_dev(I.n);
  double s = 0.0;
  // four rows per round with their loads issued together
  for (int r0 = threadIdx.x; r0 < rows; r0 += 4 * 256) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * 256;
      x[u] = r < rows ? I.diag_partial[(size_t)r * kNDiag + v] : 0.0;
    }
    s += ((x[0] + x[1]) + x[2]) + x[3];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) I.diag_out[v] = red[0];
}

// ------------------------------------------------------------ cell sort ---
// Key: the sort bin of the particle (see level_bins in particles.h).
template <typename T>
__global__ void __launch_bounds__(256)
    k_sort_key(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  __shared__ SysDev sys;
  __shared__ double cen[3 * kMaxGal];
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  const PartDev<T> p = I.p[cur[ii]];
  const gp<const T> X0 = glb((const T*)p.x[0]), X1 = glb((const T*)p.x[1]), X2 = glb((const T*)p.x[2]);
  stage(&sys, &I.sys);
  if (threadIdx.x < 3 * kMaxGal) cen[threadIdx.x] = I.centres[threadIdx.x];
  __syncthreads();
  const uint32_t lost_bin = (uint32_t)sort_bins(sys);
  const int64_t i = (int64_t)lb * 256 + threadIdx.x;
  uint32_t k = kNoKey;  // lanes past the end keep a key of their own
  if (i < p.n) {
    // flag, galaxy and position are loaded together (one round trip); a
    // lost particle's classification is computed and discarded
    const uint8_t lost = glb((const uint8_t*)p.lost)[i];
    const int g = glb((const int8_t*)p.gal)[i];
    const double x = (double)X0[i], y = (double)X1[i], z = (double)X2[i];
    const HierDev& h = sys.h[g];
    Classified c;
    classify(h, cen + 3 * g, x, y, z, c);
    k = lost_bin;
    if (!lost && c.cls != SBX_LOST) {
      const int lev = h.n_levels == 1 ? 0 : c.cls;
      const size_t n = (size_t)h.lv[lev].N;
      const int* id = lev == 0 ? c.idx[0] : (lev == 1 ? c.idx[1] : c.idx[2]);
      k = (uint32_t)(bins_before(sys, g, lev) + ((id[2] * n + id[1]) * n + id[0]));
    }
    glb(I.key)[i] = k;
  }
  // Each run of equal keys in the wavefront reserves its places in the bin
  // with one atomic from its last lane; every lane keeps its own place, so
  // the scatter needs no atomic (every lane takes part in the wave sum and
  // the shuffles: no divergent shuffles).
  const int lane = threadIdx.x & 63;
  bool tail;
  const uint32_t rank1 = wave_run_sum<uint32_t>(k, 1u, tail);  // 1-based place in the run
  uint32_t base = 0;
  if (tail && k != kNoKey)
    base = __hip_atomic_fetch_add(glb(I.count) + k, rank1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // nearest tail at or after this lane: suffix minimum of tail lane ids
  int tl = tail ? lane : 64;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t2 = __shfl_down(tl, o, 64);
    if (lane + o < 64) tl = min(tl, t2);
  }
  const uint32_t run_base = __shfl(base, tl & 63, 64);
  if (i < p.n) glb(I.rank)[i] = run_base + rank1 - 1;
}

// A particle's slot is the start of its bin (the counts scanned, global over
// all instances) plus its place in the bin from the key pass; part_base
// turns it into the instance's own slot.
//
// The reorder as a gather: k_sort_perm writes, for every particle, its
// source index at its destination slot (one scattered 4-byte stream, into
// the destination set's id array), then k_sort_gather fills each
// destination slot from its source, so the eleven streams are written
// whole, in order, and only read scattered.
template <typename T>
__global__ void __launch_bounds__(256)
    k_sort_perm(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  const int c0 = cur[ii];
  const PartDev<T> d = I.p[c0 ^ 1];
  const int64_t q = (int64_t)lb * 256 + threadIdx.x;
  if (q >= d.n) return;
  const uint32_t k = glb((const uint32_t*)I.key)[q];
  const uint32_t r = glb((const uint32_t*)I.rank)[q];
  const uint32_t j = glb((const uint32_t*)I.count)[k] + r - I.part_base;
  glb(d.id)[j] = (int32_t)q;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_sort_gather(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, Span sp) {
  const int ii = span_inst(sp, blockIdx.x);
  const int lb = blockIdx.x - sp.start[ii];
  const InstDev<T>& I = inst[ii];
  const int c0 = cur[ii];
  const PartDev<T> s = I.p[c0];
  const PartDev<T> d = I.p[c0 ^ 1];
  const int64_t j = (int64_t)lb * 256 + threadIdx.x;
  if (j >= d.n) return;
  const int64_t q = glb(d.id)[j];
  const T x0 = glb((const T*)s.x[0])[q], x1 = glb((const T*)s.x[1])[q], x2 = glb((const T*)s.x[2])[q];
  const T v0 = glb((const T*)s.v[0])[q], v1 = glb((const T*)s.v[1])[q], v2 = glb((const T*)s.v[2])[q];
  const T m = glb((const T*)s.m)[q];
  const int8_t comp = glb((const int8_t*)s.comp)[q], gal = glb((const int8_t*)s.gal)[q];
  const uint8_t lost = glb((const uint8_t*)s.lost)[q];
  const int32_t id = glb((const int32_t*)s.id)[q];
  glb((T*)d.x[0])[j] = x0;
  glb((T*)d.x[1])[j] = x1;
  glb((T*)d.x[2])[j] = x2;
  glb((T*)d.v[0])[j] = v0;
  glb((T*)d.v[1])[j] = v1;
  glb((T*)d.v[2])[j] = v2;
  glb((T*)d.m)[j] = m;
  glb(d.comp)[j] = comp;
  glb(d.gal)[j] = gal;
  glb(d.lost)[j] = lost;
  glb(d.id)[j] = id;
}

__global__ void k_flip(int* cur, int n) {
  if ((int)threadIdx.x < n) cur[threadIdx.x] ^= 1;
}


// ---------------------------------------------------------------- adjoint --
// Reverse mode of one integration cycle (see the oracle's derivation):
// lv += dt lx; mu = dt lv; lx += J mu with J the Eq. 8 second differences at
// the particle; every field the particle reads gets A^T mu on its grid (the
// Eq. 8 stencil weights transposed).  Adjoint state is kept in float64.
//
// The A^T mu contributions of a block's particles (19 cells per field) are
// summed across runs of lanes on the same cell (wavefront sums), then in an
// LDS hash table keyed like the deposit (grid slot, cell), and flushed with
// one global atomic per distinct cell; cell-sorted particles share most of
// their stencil cells.
constexpr int kAdjTableBits = 12;
constexpr int kAdjTable = 1 << kAdjTableBits;

// A key's first slot is the key modulo a prime just below the table size:
// consecutive cells take consecutive slots, so the flush, which walks the
// slots in order, hands consecutive cells to consecutive lanes and its
// global atomics coalesce (a scattering hash made them one line each and
// the flush the larger part of the kernel), while the stencil offsets
// (+-1, +-N, +-N^2 and their sums) still land on distinct slots.
constexpr uint32_t kAdjPrime = 4093u;
static_assert(kAdjPrime <= (uint32_t)kAdjTable, "slot range");

template <typename T>
struct AdjSink {
  uint32_t* tkey;
  T* tval;
  const GridsDev<T>* B;
  __device__ __forceinline__ void add(uint32_t key, double v) const {
    uint32_t h = key % kAdjPrime;
    for (int q = 0; q < 8; ++q) {
      const uint32_t old = atomicCAS(tkey + h, kNoKey, key);
      if (old == kNoKey || old == key) {
        atomicAdd(tval + h, (T)v);
        return;
      }
      h = (h + 1) & (kAdjTable - 1);
    }
    atomic_add_g(glb(slot_ptr(*B, key)), (T)v);
  }
};

// The A^T mu weights of one field at the particle (Eq. 8 stencil weights
// transposed) in the order of kAdjOff, and J mu (the field's second
// differences times mu) added to lx.  taylor = 0: only the six face
// weights are nonzero and J is not used.
constexpr int kAdjPts = 19;
template <typename T>
__device__ __forceinline__ void eq8_adjoint_weights(const T* __restrict__ F, const LevelDev& L,
                                                    const int* id, double dx, double dy, double dz,
                                                    int taylor, const double* mu, double* lx,
                                                    double* w) {
  const int sy = L.N, sz = L.N * L.N;
  const double mx = mu[0], my = mu[1], mz = mu[2];
  w[0] = mx * L.c_2l;
  w[1] = -mx * L.c_2l;
  w[2] = my * L.c_2l;
  w[3] = -my * L.c_2l;
  w[4] = mz * L.c_2lz;
  w[5] = -mz * L.c_2lz;
#pragma unroll
  for (int k = 6; k < kAdjPts; ++k) w[k] = 0.0;
  if (!taylor) return;
  const ptrdiff_t o = (ptrdiff_t)id[2] * sz + (ptrdiff_t)id[1] * sy + id[0];
  const gp<const T> P = glb(F) + o;
  const double Dx = dx - ((double)id[0] - L.half) * L.l;
  const double Dy = dy - ((double)id[1] - L.half) * L.l;
  const double Dz = dz - ((double)id[2] - L.half) * L.lz;
  // J mu from the field's second differences (symmetric)
  const double p0 = (double)P[0];
  const double hxx = ((double)P[1] + (double)P[-1] - 2.0 * p0) * L.c_l2;
  const double hyy = ((double)P[sy] + (double)P[-sy] - 2.0 * p0) * L.c_l2;
  const double hzz = ((double)P[sz] + (double)P[-sz] - 2.0 * p0) * L.c_lz2;
  const double hxy = ((double)P[1 + sy] - (double)P[-1 + sy] + (double)P[-1 - sy] - (double)P[1 - sy]) * L.c_4ll;
  const double hxz = ((double)P[1 + sz] - (double)P[-1 + sz] + (double)P[-1 - sz] - (double)P[1 - sz]) * L.c_4llz;
  const double hyz = ((double)P[sy + sz] - (double)P[-sy + sz] + (double)P[-sy - sz] - (double)P[sy - sz]) * L.c_4llz;
  lx[0] += hxx * mx + hxy * my + hxz * mz;
  lx[1] += hxy * mx + hyy * my + hyz * mz;
  lx[2] += hxz * mx + hyz * my + hzz * mz;
  // A^T mu: faces, centre, edges
  const double wx = mx * Dx * L.c_l2, wy = my * Dy * L.c_l2, wz = mz * Dz * L.c_lz2;
  w[0] += wx;
  w[1] += wx;
  w[2] += wy;
  w[3] += wy;
  w[4] += wz;
  w[5] += wz;
  w[6] = -2.0 * (wx + wy + wz);
  const double exy = (mx * Dy + my * Dx) * L.c_4ll;
  const double exz = (mx * Dz + mz * Dx) * L.c_4llz;
  const double eyz = (my * Dz + mz * Dy) * L.c_4llz;
  w[7] = exy;
  w[8] = -exy;
  w[9] = exy;
  w[10] = -exy;
  w[11] = exz;
  w[12] = -exz;
  w[13] = exz;
  w[14] = -exz;
  w[15] = eyz;
  w[16] = -eyz;
  w[17] = eyz;
  w[18] = -eyz;
}

// Cell offsets of the weights above on a grid of N cells per axis.
__device__ __forceinline__ int adj_off(int k, int N) {
  const int sy = N, sz = N * N;
  switch (k) {
    case 0: return 1;
    case 1: return -1;
    case 2: return sy;
    case 3: return -sy;
    case 4: return sz;
    case 5: return -sz;
    case 6: return 0;
    case 7: return 1 + sy;
    case 8: return -1 + sy;
    case 9: return -1 - sy;
    case 10: return 1 - sy;
    case 11: return 1 + sz;
    case 12: return -1 + sz;
    case 13: return -1 - sz;
    case 14: return 1 - sz;
    case 15: return sy + sz;
    case 16: return -sy + sz;
    case 17: return -sy - sz;
    default: return sy - sz;
  }
}

// Seed: L = sum over the selected particles of 1/2 m vz^2; dL/dvz = m vz,
// dL/dm = 1/2 vz^2 (explicit part); loss partial sums per block (fixed order).
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_init(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, int sel_comp,
               int sel_gal, double* __restrict__ lx, double* __restrict__ lv,
               double* __restrict__ gm, double* __restrict__ partial) {
  const InstDev<T>& I = inst[0];
  const PartDev<T> p = I.p[cur[0]];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    lx[3 * i] = lx[3 * i + 1] = lx[3 * i + 2] = 0.0;
    lv[3 * i] = lv[3 * i + 1] = 0.0;
    const bool sel = p.comp[i] == sel_comp && p.gal[i] == sel_gal && !p.lost[i];
    const double m = (double)p.m[i], vz = (double)p.v[2][i];
    lv[3 * i + 2] = sel ? m * vz : 0.0;
    gm[i] = sel ? 0.5 * vz * vz : 0.0;
    if (sel) acc += 0.5 * m * vz * vz;
  }
  double v[1] = {acc};
  block_sum_store<1>(v, partial + blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_step(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, GridsDev<T> Bg,
               const uint8_t* __restrict__ out, double* __restrict__ lx, double* __restrict__ lv) {
  __shared__ uint32_t tkey[kAdjTable];
  __shared__ T tval[kAdjTable];
  __shared__ double cen[3 * kMaxGal];  // read from LDS inside the galaxy loop
  // the adjoint grids' pointers, indexed by each key's slot: in LDS (taken
  // from the by-value argument with constant indices), not in scratch
  __shared__ GridsDev<T> Bs;
  const InstDev<T>& I = inst[0];
  for (int k = threadIdx.x; k < kAdjTable; k += 256) {
    tkey[k] = kNoKey;
    tval[k] = (T)0;
  }
  if (threadIdx.x < 3 * kMaxGal) cen[threadIdx.x] = I.centres[threadIdx.x];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int g = 0; g < kMaxGal; ++g)
#pragma unroll
      for (int k = 0; k < kSlots; ++k) Bs.g[g][k] = Bg.g[g][k];
  }
  __syncthreads();
  const AdjSink<T> sink{tkey, tval, &Bs};
  const PartDev<T> p = I.p[cur[0]];
  const SysDev& sys = I.sys;
  const double dt = I.dt;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // Every lane takes part in the wavefront sums below, with or without a
  // particle (act); a lane without one carries no key.
  const bool act = i < p.n && !out[i];
  double l[3] = {0.0, 0.0, 0.0}, mu[3] = {0.0, 0.0, 0.0};
  double x = 0.0, y = 0.0, z = 0.0;
  if (act) {
    l[0] = lx[3 * i];
    l[1] = lx[3 * i + 1];
    l[2] = lx[3 * i + 2];
    const double w0 = lv[3 * i] + dt * l[0], w1 = lv[3 * i + 1] + dt * l[1], w2 = lv[3 * i + 2] + dt * l[2];
    lv[3 * i] = w0;
    lv[3 * i + 1] = w1;
    lv[3 * i + 2] = w2;
    mu[0] = dt * w0;
    mu[1] = dt * w1;
    mu[2] = dt * w2;
    x = (double)p.x[0][i];
    y = (double)p.x[1][i];
    z = (double)p.x[2][i];
  }
  const GridsDev<T>& F = I.G;
  for (int g = 0; g < sys.ngal; ++g) {
    const HierDev& h = sys.h[g];
    const double* c = cen + 3 * g;
    Classified cl;
    cl.cls = SBX_LOST;
    if (act) classify(h, c, x, y, z, cl);
    const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
    const double ox = x - h.outer_c[0], oy = y - h.outer_c[1], oz = z - h.outer_c[2];
    // one field per level at most (the grid-selection rule): its slot, in
    // level order, so that lx sums the fields in the forward's order
#pragma unroll
    for (int lev = 0; lev < 3; ++lev) {  // unrolled: the cell arrays are indexed by constants
      if (lev >= h.n_levels) break;
      int slot = -1;
      if (h.n_levels == 1) {
        if (cl.cls == SBX_OUTER) slot = 0;
      } else if (lev == 0) {
        if (cl.cls == SBX_CORE) slot = 0;
      } else if (lev == 1) {
        if (cl.cls == SBX_CORE) slot = 1;
        else if (cl.cls == SBX_RING) slot = 2;
      } else {
        if (cl.cls == SBX_CORE || cl.cls == SBX_RING) slot = 3;
        else if (cl.cls == SBX_OUTER) slot = 4;
      }
      const LevelDev& L = h.lv[lev];
      const bool outer = h.n_levels > 1 && lev == 2;
      double w[kAdjPts];
      uint32_t key = kNoKey;
      if (slot >= 0) {
        key = dep_key(g, slot, L, cl.idx[lev]);
        eq8_adjoint_weights(F.g[g][slot], L, cl.idx[lev], outer ? ox : dx, outer ? oy : dy,
                            outer ? oz : dz, sys.taylor, mu, l, w);
      } else {
#pragma unroll
        for (int k = 0; k < kAdjPts; ++k) w[k] = 0.0;
      }
      // A^T mu of runs of lanes on the same cell summed across the
      // wavefront (cell-sorted particles share cells), then one table add
      // per run
      auto put = [&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const uint32_t kk = key == kNoKey ? kNoKey : (uint32_t)((int)key + adj_off(k, L.N));
        bool tail;
        const double sum = wave_run_sum<double>(kk, w[k], tail);
        if (tail && kk != kNoKey) sink.add(kk, sum);
      };
      put(std::integral_constant<int, 0>());
      put(std::integral_constant<int, 1>());
      put(std::integral_constant<int, 2>());
      put(std::integral_constant<int, 3>());
      put(std::integral_constant<int, 4>());
      put(std::integral_constant<int, 5>());
      if (sys.taylor) {
        put(std::integral_constant<int, 6>());
        put(std::integral_constant<int, 7>());
        put(std::integral_constant<int, 8>());
        put(std::integral_constant<int, 9>());
        put(std::integral_constant<int, 10>());
        put(std::integral_constant<int, 11>());
        put(std::integral_constant<int, 12>());
        put(std::integral_constant<int, 13>());
        put(std::integral_constant<int, 14>());
        put(std::integral_constant<int, 15>());
        put(std::integral_constant<int, 16>());
        put(std::integral_constant<int, 17>());
        put(std::integral_constant<int, 18>());
      }
    }
  }
  if (act) {
    lx[3 * i] = l[0];
    lx[3 * i + 1] = l[1];
    lx[3 * i + 2] = l[2];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kAdjTable; k += 256) {
    const uint32_t key = tkey[k];
    if (key != kNoKey) atomic_add_g(glb(slot_ptr(Bs, key)), tval[k]);
  }
}

template <typename T>
__device__ __forceinline__ const T* cell_ptr(const T* grid, const LevelDev& L, const int* i) {
  return grid + ((size_t)i[2] * L.N + i[1]) * L.N + i[0];
}

// Mass gradient: the adjoint potential psi of every grid a particle feeds,
// read at its source cell (the transpose of the nearest-grid-point deposit).
template <typename T>
__global__ void __launch_bounds__(256)
    k_adj_gather(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, GridsDev<T> Pg,
                 const uint8_t* __restrict__ out, double* __restrict__ gm) {
  const InstDev<T>& I = inst[0];
  const PartDev<T> p = I.p[cur[0]];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n || out[i]) return;
  const int g = p.gal[i];
  const HierDev& h = I.sys.h[g];
  Classified c;
  classify(h, I.centres + 3 * g, (double)p.x[0][i], (double)p.x[1][i], (double)p.x[2][i], c);
  double s = 0.0;
  auto at = [&](int slot, int lev) { return (double)*cell_ptr(Pg.g[g][slot], h.lv[lev], c.idx[lev]); };
  if (h.n_levels == 1) {
    if (c.cls == SBX_OUTER) s = at(0, 0);
  } else if (c.cls == SBX_CORE) {
    s = at(0, 0) + at(2, 1) + at(4, 2);
  } else if (c.cls == SBX_RING) {
    s = at(1, 1) + at(2, 1) + at(4, 2);
  } else if (c.cls == SBX_OUTER) {
    s = at(3, 2) + at(4, 2);
  }
  gm[i] += s;
}

// ------------------------------------------------------------- readouts ---
template <typename T>
__global__ void k_indices(const InstDev<T>* __restrict__ inst, const int* __restrict__ cur, int g,
                          int level, int32_t* __restrict__ idx, int8_t* __restrict__ cls) {
  const InstDev<T>& I = inst[0];
  const PartDev<T> p = I.p[cur[0]];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  Classified c;
  classify(I.sys.h[g], I.centres + 3 * g, (double)p.x[0][i], (double)p.x[1][i], (double)p.x[2][i], c);
  if (idx) {
    idx[3 * i] = c.idx[level][0];
    idx[3 * i + 1] = c.idx[level][1];
    idx[3 * i + 2] = c.idx[level][2];
  }
  if (cls) cls[i] = (int8_t)c.cls;
}

template <typename T>
__global__ void k_zero(T* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ s, B* __restrict__ d, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = (B)s[i];
}

template <typename T>
__global__ void k_split3(const double* __restrict__ s, T* x0, T* x1, T* x2, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x0[i] = (T)s[3 * i];
    x1[i] = (T)s[3 * i + 1];
    x2[i] = (T)s[3 * i + 2];
  }
}

template <typename T>
__global__ void k_join3(const T* x0, const T* x1, const T* x2, double* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    d[3 * i] = (double)x0[i];
    d[3 * i + 1] = (double)x1[i];
    d[3 * i + 2] = (double)x2[i];
  }
}

__global__ void k_iota(int32_t* id, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    id[i] = (int32_t)i;
}

template <typename A>
__global__ void k_unpermute(const A* __restrict__ src, const int32_t* __restrict__ id,
                            A* __restrict__ dst, int64_t n, int width) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = id[i];
    for (int w = 0; w < width; ++w) dst[j * width + w] = src[i * width + w];
  }
}

// ------------------------------------------------------------- launchers --
template <typename T>
sbx_status launch_zero(T* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_zero<T>), dim3(2048), dim3(256), 0, s, p, n);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

static sbx_status check_span(const std::vector<InstInfo>& info) {
  if (info.empty() || (int)info.size() > kMaxInst) {
    set_error("1 to 32 instances per launch");
    return SBX_EINVAL;
  }
  return SBX_OK;
}

template <typename T>
sbx_status launch_zero_grids(const InstDev<T>* inst, const std::vector<InstInfo>& info, hipStream_t s) {
  SBX_TRY(check_span(info));
  const Span sp = make_span(info, blocks_grid);
  hipLaunchKernelGGL((k_zero_grids<T>), dim3(sp.start[sp.ninst]), dim3(256), 0, s, inst, sp);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_zero_and_centres(const InstDev<T>* inst, const std::vector<InstInfo>& info,
                                   hipStream_t s) {
  SBX_TRY(check_span(info));
  const Span sp = make_span(info, blocks_grid);
  hipLaunchKernelGGL((k_zero_centres<T>), dim3(sp.start[sp.ninst]), dim3(256), 0, s, inst, sp);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_centres(const InstDev<T>* inst, const int* cur, const std::vector<InstInfo>& info,
                          bool from_com, hipStream_t s, bool density) {
  SBX_TRY(check_span(info));
  if (!from_com) {
    const Span sp = make_span(info, blocks_red);
    hipLaunchKernelGGL((k_pre<T>), dim3(sp.start[sp.ninst]), dim3(256), 0, s, inst, cur, sp);
  }
  bool any_dm = false;
  for (const InstInfo& f : info) any_dm = any_dm || f.dm_elems > 0;
  if (density && any_dm) {
    const unsigned ni = (unsigned)info.size();
    const Span sz = make_span(info, blocks_dm);
    const Span sr = make_span(info, blocks_red);
    const Span sq = make_span(info, blocks_particles);
    hipLaunchKernelGGL((k_dm_zero<T>), dim3(sz.start[sz.ninst]), dim3(256), 0, s, inst, sz);
    hipLaunchKernelGGL((k_dm_hist<T>), dim3(sq.start[sq.ninst]), dim3(256), 0, s, inst, cur, sq);
    hipLaunchKernelGGL((k_dm_arg1<T>), dim3(kArgParts, kMaxGal, ni), dim3(256), 0, s, inst);
    hipLaunchKernelGGL((k_dm_arg2<T>), dim3(kMaxGal, ni), dim3(256), 0, s, inst);
    hipLaunchKernelGGL((k_dm_window<T>), dim3(sr.start[sr.ninst]), dim3(256), 0, s, inst, cur, sr);
  }
  hipLaunchKernelGGL((k_centres<T>), dim3((unsigned)info.size()), dim3(256), 0, s, inst, from_com ? 1 : 0,
                     density ? 1 : 0);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_deposit(const InstDev<T>* inst, const int* cur, const std::vector<InstInfo>& info,
                          hipStream_t s) {
  SBX_TRY(check_span(info));
  const Span sp = make_span(info, blocks_deposit);
  if (info[0].fix) {
    hipLaunchKernelGGL((k_deposit<T, true>), dim3(sp.start[sp.ninst]), dim3(256), 0, s, inst, cur, sp);
    const Span sg = make_span(info, blocks_grid);
    hipLaunchKernelGGL((k_fix_convert<T>), dim3(sg.start[sg.ninst]), dim3(256), 0, s, inst, sg);
  } else {
    hipLaunchKernelGGL((k_deposit<T, false>), dim3(sp.start[sp.ninst]), dim3(256), 0, s, inst, cur, sp);
  }
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_force(const InstDev<T>* inst, const int* cur, const std::vector<InstInfo>& info,
                        int mode, hipStream_t s) {
  SBX_TRY(check_span(info));
  const Span sp = make_span(info, blocks_force);
  const dim3 g(sp.start[sp.ninst]), b(256);
#define SBX_FORCE(M)                                                             \
  case M:                                                                        \
    hipLaunchKernelGGL((k_force<T, M>), g, b, 0, s, inst, cur, sp);             \
    break;
  switch (mode) {
    SBX_FORCE(1)
    SBX_FORCE(2)
    SBX_FORCE(4)
    SBX_FORCE(5)
    SBX_FORCE(6)
    default:
      set_error("bad force mode");
      return SBX_EINVAL;
  }
#undef SBX_FORCE
  if (mode & 4)
    hipLaunchKernelGGL((k_diag_final<T>), dim3(kNDiag, (unsigned)info.size()), dim3(256), 0, s, inst);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_sort(const InstDev<T>* inst, int* cur, const std::vector<InstInfo>& info,
                       uint32_t* counts, size_t total_counts, uint32_t* tmp, hipStream_t s) {
  SBX_TRY(check_span(info));
  const Span sp = make_span(info, blocks_particles);
  SBX_TRY(launch_zero<uint32_t>(counts, total_counts, s));
  hipLaunchKernelGGL((k_sort_key<T>), dim3(sp.start[sp.ninst]), dim3(256), 0, s, inst, cur, sp);
  SBX_HIP(hipGetLastError());
  SBX_TRY(exclusive_scan_u32(counts, total_counts, tmp, s));
  const Span sq = make_span(info, blocks_sort);
  hipLaunchKernelGGL((k_sort_perm<T>), dim3(sq.start[sq.ninst]), dim3(256), 0, s, inst, cur, sq);
  hipLaunchKernelGGL((k_sort_gather<T>), dim3(sq.start[sq.ninst]), dim3(256), 0, s, inst, cur, sq);
  hipLaunchKernelGGL(k_flip, dim3(1), dim3(64), 0, s, cur, (int)info.size());
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_indices(const InstDev<T>* inst, const int* cur, int64_t n, int galaxy, int level,
                          int32_t* idx, int8_t* cls, hipStream_t s) {
  if (n == 0) return SBX_OK;
  hipLaunchKernelGGL((k_indices<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, inst, cur,
                     galaxy, level, idx, cls);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}


template <typename T>
sbx_status launch_adj_init(const InstDev<T>* inst, const int* cur, int64_t n, int sel_comp,
                           int sel_gal, double* lx, double* lv, double* gm, double* partial,
                           double* loss, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_init<T>), dim3(kRedBlocks), dim3(256), 0, s, inst, cur, sel_comp, sel_gal,
                     lx, lv, gm, partial);
  hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(256), 0, s, partial, kRedBlocks, loss);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_adj_step(const InstDev<T>* inst, const int* cur, int64_t n, const GridsDev<T>& B,
                           const uint8_t* out, double* lx, double* lv, hipStream_t s) {
  if (n == 0) return SBX_OK;
  hipLaunchKernelGGL((k_adj_step<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, inst, cur, B,
                     out, lx, lv);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_adj_gather(const InstDev<T>* inst, const int* cur, int64_t n, const GridsDev<T>& P,
                             const uint8_t* out, double* gm, hipStream_t s) {
  if (n == 0) return SBX_OK;
  hipLaunchKernelGGL((k_adj_gather<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, inst, cur, P,
                     out, gm);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

// First particle (lowest index) whose inputs are not acceptable: non-finite
// or negative mass, non-finite position or velocity, component outside
// 0..kNComp-1, galaxy outside 0..ngal-1.  *bad stays at its initial value
// (all ones) when every particle is acceptable.
__global__ void k_validate_particles(const double* __restrict__ x, const double* __restrict__ v,
                                     const double* __restrict__ m, const int8_t* __restrict__ comp,
                                     const int8_t* __restrict__ gal, int64_t n, int ngal,
                                     unsigned long long* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool ok = isfinite(m[i]) && m[i] >= 0.0 && comp[i] >= 0 && comp[i] < kNComp && gal[i] >= 0 &&
              gal[i] < ngal;
#pragma unroll
    for (int k = 0; k < 3; ++k) ok = ok && isfinite(x[3 * i + k]) && isfinite(v[3 * i + k]);
    if (!ok) atomicMin(bad, (unsigned long long)i);
  }
}

sbx_status launch_validate_particles(const double* x, const double* v, const double* m,
                                     const int8_t* comp, const int8_t* gal, int64_t n, int ngal,
                                     unsigned long long* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_particles, dim3(2048), dim3(256), 0, s, x, v, m, comp, gal, n, ngal, bad);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
__global__ void k_validate_soa(const T* __restrict__ x, const T* __restrict__ v,
                               const T* __restrict__ m, const int8_t* __restrict__ comp,
                               const int8_t* __restrict__ gal, int64_t n, int ngal,
                               unsigned long long* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool ok = isfinite((double)m[i]) && m[i] >= (T)0 && comp[i] >= 0 && comp[i] < kNComp &&
              gal[i] >= 0 && gal[i] < ngal;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      ok = ok && isfinite((double)x[k * n + i]) && isfinite((double)v[k * n + i]);
    if (!ok) atomicMin(bad, (unsigned long long)i);
  }
}

template <typename T>
sbx_status launch_validate_soa(const T* x, const T* v, const T* m, const int8_t* comp,
                               const int8_t* gal, int64_t n, int ngal, unsigned long long* bad,
                               hipStream_t s) {
  hipLaunchKernelGGL((k_validate_soa<T>), dim3(2048), dim3(256), 0, s, x, v, m, comp, gal, n, ngal, bad);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}
template sbx_status launch_validate_soa<float>(const float*, const float*, const float*, const int8_t*,
                                               const int8_t*, int64_t, int, unsigned long long*,
                                               hipStream_t);
template sbx_status launch_validate_soa<double>(const double*, const double*, const double*,
                                                const int8_t*, const int8_t*, int64_t, int,
                                                unsigned long long*, hipStream_t);

template <typename T>
sbx_status launch_mass_max(const T* m, int64_t n, unsigned long long* out, hipStream_t s) {
  SBX_HIP(hipMemsetAsync(out, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL((k_mass_max<T>), dim3(1024), dim3(256), 0, s, m, n, out);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}
template sbx_status launch_mass_max<float>(const float*, int64_t, unsigned long long*, hipStream_t);
template sbx_status launch_mass_max<double>(const double*, int64_t, unsigned long long*, hipStream_t);

sbx_status launch_iota(int32_t* id, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(2048), dim3(256), 0, s, id, n);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename A>
sbx_status launch_unpermute(const A* src, const int32_t* id, A* dst, int64_t n, int width,
                            hipStream_t s) {
  hipLaunchKernelGGL((k_unpermute<A>), dim3(2048), dim3(256), 0, s, src, id, dst, n, width);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_convert_in(const double* src, T* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, T>), dim3(2048), dim3(256), 0, s, src, dst, n);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_convert_out(const T* src, double* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<T, double>), dim3(2048), dim3(256), 0, s, src, dst, n);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_split3(const double* src, T* x0, T* x1, T* x2, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_split3<T>), dim3(2048), dim3(256), 0, s, src, x0, x1, x2, n);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status launch_join3(const T* x0, const T* x1, const T* x2, double* dst, int64_t n,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_join3<T>), dim3(2048), dim3(256), 0, s, x0, x1, x2, dst, n);
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

#define SBX_INST(T)                                                                              \
  template sbx_status launch_zero<T>(T*, size_t, hipStream_t);                                   \
  template sbx_status launch_zero_grids<T>(const InstDev<T>*, const std::vector<InstInfo>&,      \
                                           hipStream_t);                                         \
  template sbx_status launch_zero_and_centres<T>(const InstDev<T>*, const std::vector<InstInfo>&, \
                                                 hipStream_t);                                   \
  template sbx_status launch_centres<T>(const InstDev<T>*, const int*,                           \
                                        const std::vector<InstInfo>&, bool, hipStream_t, bool);  \
  template sbx_status launch_deposit<T>(const InstDev<T>*, const int*,                           \
                                        const std::vector<InstInfo>&, hipStream_t);              \
  template sbx_status launch_force<T>(const InstDev<T>*, const int*, const std::vector<InstInfo>&, \
                                      int, hipStream_t);                                         \
  template sbx_status launch_sort<T>(const InstDev<T>*, int*, const std::vector<InstInfo>&,      \
                                     uint32_t*, size_t, uint32_t*, hipStream_t);                 \
  template sbx_status launch_indices<T>(const InstDev<T>*, const int*, int64_t, int, int,        \
                                        int32_t*, int8_t*, hipStream_t);                         \
  template sbx_status launch_adj_init<T>(const InstDev<T>*, const int*, int64_t, int, int,       \
                                         double*, double*, double*, double*, double*,            \
                                         hipStream_t);                                           \
  template sbx_status launch_adj_step<T>(const InstDev<T>*, const int*, int64_t,                 \
                                         const GridsDev<T>&, const uint8_t*, double*, double*,   \
                                         hipStream_t);                                           \
  template sbx_status launch_adj_gather<T>(const InstDev<T>*, const int*, int64_t,               \
                                           const GridsDev<T>&, const uint8_t*, double*,          \
                                           hipStream_t);                                         \
  template sbx_status launch_convert_in<T>(const double*, T*, size_t, hipStream_t);              \
  template sbx_status launch_convert_out<T>(const T*, double*, size_t, hipStream_t);             \
  template sbx_status launch_split3<T>(const double*, T*, T*, T*, int64_t, hipStream_t);         \
  template sbx_status launch_join3<T>(const T*, const T*, const T*, double*, int64_t, hipStream_t);
SBX_INST(float)
SBX_INST(double)
#undef SBX_INST
template sbx_status launch_zero<uint32_t>(uint32_t*, size_t, hipStream_t);
template sbx_status launch_zero<uint8_t>(uint8_t*, size_t, hipStream_t);
template sbx_status launch_unpermute<double>(const double*, const int32_t*, double*, int64_t, int, hipStream_t);
template sbx_status launch_unpermute<int32_t>(const int32_t*, const int32_t*, int32_t*, int64_t, int, hipStream_t);
template sbx_status launch_unpermute<int8_t>(const int8_t*, const int32_t*, int8_t*, int64_t, int, hipStream_t);
template sbx_status launch_unpermute<uint8_t>(const uint8_t*, const int32_t*, uint8_t*, int64_t, int, hipStream_t);

}  // namespace sbx
