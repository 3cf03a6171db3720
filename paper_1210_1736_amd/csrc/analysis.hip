// Disc diagnostics of the paper's analysis (Sec. 4.2 and 5.2-5.4): heat of
// the disc with the mean circular velocity from radial bins of equal
// particle numbers, RMS thickness per bin, vertical density profile and
// velocity dispersions in an annulus.  The radial order comes from a stable
// least-significant-digit radix sort of the FP64 radii (ties keep the
// caller's particle order).  Every sum except the vertical profile is
// reduced in a fixed order.
#include "ctx.h"

using namespace sbx;

namespace {

constexpr int kRsTile = 1024;  // elements per radix block (one wavefront, 16 chunks)
constexpr int kRsChunks = kRsTile / 64;
constexpr int kMaxBins = 2048;
constexpr int kMaxZ = 1024;
constexpr int kAnBlocks = 512;  // blocks of the heat / annulus pass
// per-block partial row: heat, annulus count, sum vR, vR^2, vphi, vphi^2, vz, vz^2
constexpr int kAnVals = 8;

// ------------------------------------------------------------- selection --
// flag (caller order) of the disc particles
template <typename T>
__global__ void k_disc_flags(PartDev<T> p, int comp, int gal, uint32_t* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[p.id[i]] = (p.comp[i] == comp && p.gal[i] == gal && !p.lost[i]) ? 1u : 0u;
}

// compact arrays in caller order: position relative to the centre, velocity,
// mass; pos holds the exclusive scan of the flags
template <typename T>
__global__ void k_disc_compact(PartDev<T> p, int comp, int gal, const uint32_t* __restrict__ pos,
                               const double* __restrict__ centre, double* __restrict__ d3,
                               double* __restrict__ v3, double* __restrict__ m1) {
  const double cx = centre[0], cy = centre[1], cz = centre[2];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!(p.comp[i] == comp && p.gal[i] == gal && !p.lost[i])) continue;
    const uint32_t k = pos[p.id[i]];
    d3[3 * k] = (double)p.x[0][i] - cx;
    d3[3 * k + 1] = (double)p.x[1][i] - cy;
    d3[3 * k + 2] = (double)p.x[2][i] - cz;
    v3[3 * k] = (double)p.v[0][i];
    v3[3 * k + 1] = (double)p.v[1][i];
    v3[3 * k + 2] = (double)p.v[2][i];
    m1[k] = (double)p.m[i];
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum of nv values over a 256-thread block into out[0..nv).
template <int NV>
__device__ __forceinline__ void block_rows(const double* vals, double* out) {
  __shared__ double red[4][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wsum(vals[k]);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += blockDim.x) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// sums of m and m v over the disc (block partials)
__global__ void __launch_bounds__(256)
    k_disc_bulk(const double* __restrict__ v3, const double* __restrict__ m1, int64_t n,
                double* __restrict__ part) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double m = m1[i];
    a[0] += m;
    a[1] += m * v3[3 * i];
    a[2] += m * v3[3 * i + 1];
    a[3] += m * v3[3 * i + 2];
  }
  block_rows<4>(a, part + 4 * (size_t)blockIdx.x);
}

// column sums of rows x nv partials (one block per column, fixed order)
__global__ void __launch_bounds__(256)
    k_columns(const double* __restrict__ part, int rows, int nv, double* __restrict__ out) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) s += part[(size_t)r * nv + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// cylindrical quantities relative to the disc's mean velocity; radix key of R
__global__ void k_disc_cyl(const double* __restrict__ d3, const double* __restrict__ v3,
                           const double* __restrict__ bulk, int64_t n, double* __restrict__ R,
                           double* __restrict__ vR, double* __restrict__ vphi,
                           double* __restrict__ vz, uint64_t* __restrict__ key,
                           uint32_t* __restrict__ val) {
#pragma clang fp contract(off)
  const double M = bulk[0];
  const double bx = bulk[1] / M, by = bulk[2] / M, bz = bulk[3] / M;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double dx = d3[3 * i], dy = d3[3 * i + 1];
    const double ux = v3[3 * i] - bx, uy = v3[3 * i + 1] - by, uz = v3[3 * i + 2] - bz;
    const double r = sqrt(dx * dx + dy * dy);
    R[i] = r;
    vR[i] = r > 0.0 ? (dx * ux + dy * uy) / r : 0.0;
    vphi[i] = r > 0.0 ? (dx * uy - dy * ux) / r : 0.0;
    vz[i] = uz;
    key[i] = (uint64_t)__double_as_longlong(r);  // R >= 0: bit order is value order
    val[i] = (uint32_t)i;
  }
}

// ------------------------------------------------------------ radix sort --
__device__ __forceinline__ int digit_of(uint64_t k, int shift) { return (int)((k >> shift) & 0xFF); }

// per-tile histogram of one 8-bit digit, stored digit-major: cnt[d * nb + b]
__global__ void __launch_bounds__(64)
    k_rs_hist(const uint64_t* __restrict__ key, int64_t n, int shift, int nb, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[256];
  for (int d = threadIdx.x; d < 256; d += 64) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int c = 0; c < kRsChunks; ++c) {
    const int64_t e = base + c * 64 + threadIdx.x;
    if (e < n) atomicAdd(h + digit_of(key[e], shift), 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += 64) cnt[(size_t)d * nb + blockIdx.x] = h[d];
}

// stable scatter: within a tile, elements keep their order (chunks in
// order, lanes in order: rank among equal digits by ballots)
__global__ void __launch_bounds__(64)
    k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, int64_t n,
                 int shift, int nb, const uint32_t* __restrict__ off, uint64_t* __restrict__ kout,
                 uint32_t* __restrict__ vout) {
  __shared__ uint32_t o[256];
  const int lane = threadIdx.x;
  for (int d = lane; d < 256; d += 64) o[d] = off[(size_t)d * nb + blockIdx.x];
  __syncthreads();
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int c = 0; c < kRsChunks; ++c) {
    const int64_t e = base + c * 64 + lane;
    const bool ok = e < n;
    const uint64_t k = ok ? kin[e] : 0ull;
    const int d = digit_of(k, shift);
    uint64_t match = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(ok && bit);
      match &= bit ? bb : ~bb;
    }
    const int rank = __popcll(match & lt);
    const uint32_t start = ok ? o[d] : 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (ok) {
      kout[start + rank] = k;
      vout[start + rank] = vin[e];
      if (rank == 0) o[d] = start + (uint32_t)__popcll(match);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ------------------------------------------------------------------- bins --
// one block per bin: mean R, mean v_phi, RMS z over the bin's range of the
// sorted order (bin k: n / nbins items, plus one for k < n % nbins)
__global__ void __launch_bounds__(256)
    k_disc_bins(const uint32_t* __restrict__ order, int64_t n, int nbins, const double* __restrict__ R,
                const double* __restrict__ vphi, const double* __restrict__ d3,
                double* __restrict__ bin_r, double* __restrict__ bin_vc, double* __restrict__ bin_rz) {
  const int k = blockIdx.x;
  const int64_t q = n / nbins, r = n % nbins;
  const int64_t s0 = k * q + (k < r ? k : r);
  const int64_t s1 = s0 + q + (k < r ? 1 : 0);
  double a[3] = {0.0, 0.0, 0.0};
  for (int64_t j = s0 + threadIdx.x; j < s1; j += 256) {
    const uint32_t i = order[j];
    const double z = d3[3 * (size_t)i + 2];
    a[0] += R[i];
    a[1] += vphi[i];
    a[2] += z * z;
  }
  __shared__ double out[3];
  block_rows<3>(a, out);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double c = (double)(s1 - s0);
    bin_r[k] = c > 0 ? out[0] / c : 0.0;
    bin_vc[k] = c > 0 ? out[1] / c : 0.0;
    bin_rz[k] = c > 0 ? sqrt(out[2] / c) : 0.0;
  }
}

// heat with the interpolated circular velocity; annulus sums; z profile
__global__ void __launch_bounds__(256)
    k_disc_heat(int64_t n, int nbins, const double* __restrict__ bin_r, const double* __restrict__ bin_vc,
                const double* __restrict__ R, const double* __restrict__ vR,
                const double* __restrict__ vphi, const double* __restrict__ vz,
                const double* __restrict__ d3, const double* __restrict__ m1, double lo, double hi,
                int nz, double zmax, double* __restrict__ part, double* __restrict__ zpart) {
  extern __shared__ double sh[];  // bin_r, bin_vc (nbins each), then nz profile bins
  double* br = sh;
  double* bv = sh + nbins;
  double* hz = sh + 2 * nbins;
  for (int k = threadIdx.x; k < nbins; k += 256) {
    br[k] = bin_r[k];
    bv[k] = bin_vc[k];
  }
  for (int k = threadIdx.x; k < nz; k += 256) hz[k] = 0.0;
  __syncthreads();
  const double dz = 2.0 * zmax / nz;
  double a[kAnVals] = {};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double r = R[i], m = m1[i];
    // vbar_c(r): linear between the bins' mean radii, constant beyond the ends
    double vc;
    if (r <= br[0]) {
      vc = bv[0];
    } else if (r >= br[nbins - 1]) {
      vc = bv[nbins - 1];
    } else {
      int lo_k = 0, hi_k = nbins - 1;  // br[lo_k] < r < br[hi_k]
      while (hi_k - lo_k > 1) {
        const int mid = (lo_k + hi_k) >> 1;
        if (br[mid] <= r) lo_k = mid;
        else hi_k = mid;
      }
      const double t = (r - br[lo_k]) / (br[hi_k] - br[lo_k]);
      vc = bv[lo_k] + t * (bv[hi_k] - bv[lo_k]);
    }
    const double a_r = vR[i], a_p = vphi[i], a_z = vz[i];
    const double dp = a_p - vc;
    a[0] += 0.5 * m * ((a_r * a_r + dp * dp) + a_z * a_z);
    if (r >= lo && r < hi) {
      a[1] += 1.0;
      a[2] += a_r;
      a[3] += a_r * a_r;
      a[4] += a_p;
      a[5] += a_p * a_p;
      a[6] += a_z;
      a[7] += a_z * a_z;
      const double z = d3[3 * i + 2];
      if (z >= -zmax && z < zmax) {
        int k = (int)floor((z + zmax) / dz);
        k = k < nz - 1 ? k : nz - 1;
        atomicAdd(hz + k, m);
      }
    }
  }
  block_rows<kAnVals>(a, part + (size_t)kAnVals * blockIdx.x);
  __syncthreads();
  for (int k = threadIdx.x; k < nz; k += 256) zpart[(size_t)blockIdx.x * nz + k] = hz[k];
}

template <typename T>
PartDev<T> live_set(sbx_ctx* c) {
  const PSet& q = c->set[c->cur];
  PartDev<T> p;
  for (int k = 0; k < 3; ++k) {
    p.x[k] = (T*)q.x[k];
    p.v[k] = (T*)q.v[k];
  }
  p.m = (T*)q.m;
  p.comp = q.comp;
  p.gal = q.gal;
  p.lost = q.lost;
  p.id = q.id;
  p.n = c->n;
  return p;
}

// Device buffers of a prepared disc: compact arrays in caller order and the
// radial order.  Freed together.
struct Disc {
  std::vector<void*> allocs;
  int64_t n = 0;
  double *d3 = nullptr, *v3 = nullptr, *m1 = nullptr, *bulk = nullptr;
  double *R = nullptr, *vR = nullptr, *vphi = nullptr, *vz = nullptr;
  uint64_t* key = nullptr;    // sorted radius keys (FP64 bits)
  uint32_t* order = nullptr;  // compact index of the sorted positions
  sbx_status alloc(void** p, size_t bytes) {
    const sbx_status r = dev_alloc(p, bytes ? bytes : 8);
    if (r == SBX_OK) allocs.push_back(*p);
    return r;
  }
  ~Disc() {
    for (void* q : allocs) (void)hipFree(q);
  }
};

// Select the disc (caller order), centre it on the galaxy, take velocities
// relative to its mean, compute cylindrical quantities, sort by radius.
template <typename T>
sbx_status disc_prepare(sbx_ctx* c, int comp, int galaxy, Disc& D) {
  const int64_t n = c->n;
  hipStream_t s = c->stream;
  const PartDev<T> p = live_set<T>(c);
  uint32_t *flag = nullptr, *tmp = nullptr;
  SBX_TRY(D.alloc((void**)&flag, sizeof(uint32_t) * (n + 1)));
  SBX_TRY(D.alloc((void**)&tmp, sizeof(uint32_t) * scan_tmp_elems(n + 1)));
  SBX_TRY(launch_zero<uint32_t>(flag, n + 1, s));
  hipLaunchKernelGGL((k_disc_flags<T>), dim3(1024), dim3(256), 0, s, p, comp, galaxy, flag);
  SBX_TRY(exclusive_scan_u32(flag, n + 1, tmp, s));
  uint32_t nd32 = 0;
  SBX_HIP(hipMemcpyAsync(&nd32, flag + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  SBX_HIP(hipStreamSynchronize(s));
  const int64_t nd = nd32;
  D.n = nd;
  if (nd == 0) {
    set_error("no live particles of the requested disc component");
    return SBX_ESTATE;
  }
  // centre of the galaxy's grids at the last solve (else its given centre)
  double cen[3];
  for (int k = 0; k < 3; ++k) cen[k] = c->hh[galaxy].centre[k];
  if (c->solved) SBX_HIP(hipMemcpy(cen, c->centres + 3 * galaxy, sizeof(cen), hipMemcpyDeviceToHost));
  double *dcen = nullptr, *part = nullptr;
  SBX_TRY(D.alloc((void**)&dcen, sizeof(cen)));
  SBX_HIP(hipMemcpyAsync(dcen, cen, sizeof(cen), hipMemcpyHostToDevice, s));
  SBX_TRY(D.alloc((void**)&D.d3, sizeof(double) * 3 * nd));
  SBX_TRY(D.alloc((void**)&D.v3, sizeof(double) * 3 * nd));
  SBX_TRY(D.alloc((void**)&D.m1, sizeof(double) * nd));
  hipLaunchKernelGGL((k_disc_compact<T>), dim3(1024), dim3(256), 0, s, p, comp, galaxy, flag, dcen, D.d3,
                     D.v3, D.m1);
  SBX_TRY(D.alloc((void**)&part, sizeof(double) * 1024 * 4));
  SBX_TRY(D.alloc((void**)&D.bulk, sizeof(double) * 4));
  hipLaunchKernelGGL(k_disc_bulk, dim3(1024), dim3(256), 0, s, D.v3, D.m1, nd, part);
  hipLaunchKernelGGL(k_columns, dim3(4), dim3(256), 0, s, part, 1024, 4, D.bulk);
  uint64_t* kb = nullptr;
  uint32_t *vb = nullptr, *cnt = nullptr, *ctmp = nullptr;
  SBX_TRY(D.alloc((void**)&D.R, sizeof(double) * nd));
  SBX_TRY(D.alloc((void**)&D.vR, sizeof(double) * nd));
  SBX_TRY(D.alloc((void**)&D.vphi, sizeof(double) * nd));
  SBX_TRY(D.alloc((void**)&D.vz, sizeof(double) * nd));
  SBX_TRY(D.alloc((void**)&D.key, sizeof(uint64_t) * nd));
  SBX_TRY(D.alloc((void**)&kb, sizeof(uint64_t) * nd));
  SBX_TRY(D.alloc((void**)&D.order, sizeof(uint32_t) * nd));
  SBX_TRY(D.alloc((void**)&vb, sizeof(uint32_t) * nd));
  hipLaunchKernelGGL(k_disc_cyl, dim3(1024), dim3(256), 0, s, D.d3, D.v3, D.bulk, nd, D.R, D.vR, D.vphi,
                     D.vz, D.key, D.order);
  const int nb = (int)((nd + kRsTile - 1) / kRsTile);
  const size_t ncnt = (size_t)256 * nb;
  SBX_TRY(D.alloc((void**)&cnt, sizeof(uint32_t) * ncnt));
  SBX_TRY(D.alloc((void**)&ctmp, sizeof(uint32_t) * scan_tmp_elems(ncnt)));
  uint64_t* ka = D.key;
  uint32_t* va = D.order;
  for (int shift = 0; shift < 64; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(64), 0, s, ka, nd, shift, nb, cnt);
    SBX_TRY(exclusive_scan_u32(cnt, ncnt, ctmp, s));
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(64), 0, s, ka, va, nd, shift, nb, cnt, kb, vb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  D.key = ka;  // eight passes: the sorted data is back in the first buffers
  D.order = va;
  SBX_HIP(hipGetLastError());
  return SBX_OK;
}

template <typename T>
sbx_status disc_t(sbx_ctx* c, const sbx_disc_query* qy, sbx_disc_result* res, double* bin_r,
                  double* bin_vc, double* bin_rms_z, double* rho_z) {
  hipStream_t s = c->stream;
  Disc D;
  auto body = [&]() -> sbx_status {
    SBX_TRY(disc_prepare<T>(c, qy->comp, qy->galaxy, D));
    const int64_t nd = D.n;
    res->n_disc = nd;
    const int nbins = qy->n_bins;
    double *br = nullptr, *bv = nullptr, *bz = nullptr, *apart = nullptr, *zpart = nullptr,
           *asum = nullptr, *zsum = nullptr;
    SBX_TRY(D.alloc((void**)&br, sizeof(double) * nbins));
    SBX_TRY(D.alloc((void**)&bv, sizeof(double) * nbins));
    SBX_TRY(D.alloc((void**)&bz, sizeof(double) * nbins));
    hipLaunchKernelGGL(k_disc_bins, dim3(nbins), dim3(256), 0, s, D.order, nd, nbins, D.R, D.vphi, D.d3, br,
                       bv, bz);
    SBX_TRY(D.alloc((void**)&apart, sizeof(double) * kAnBlocks * kAnVals));
    SBX_TRY(D.alloc((void**)&zpart, sizeof(double) * kAnBlocks * qy->n_z));
    SBX_TRY(D.alloc((void**)&asum, sizeof(double) * kAnVals));
    SBX_TRY(D.alloc((void**)&zsum, sizeof(double) * qy->n_z));
    const size_t shb = sizeof(double) * (2 * (size_t)nbins + qy->n_z);
    hipLaunchKernelGGL(k_disc_heat, dim3(kAnBlocks), dim3(256), shb, s, nd, nbins, br, bv, D.R, D.vR, D.vphi,
                       D.vz, D.d3, D.m1, qy->annulus[0], qy->annulus[1], qy->n_z, qy->z_max, apart, zpart);
    hipLaunchKernelGGL(k_columns, dim3(kAnVals), dim3(256), 0, s, apart, kAnBlocks, kAnVals, asum);
    hipLaunchKernelGGL(k_columns, dim3(qy->n_z), dim3(256), 0, s, zpart, kAnBlocks, qy->n_z, zsum);
    SBX_HIP(hipGetLastError());
    double a[kAnVals], b4[4];
    std::vector<double> z(qy->n_z);
    SBX_HIP(hipMemcpyAsync(a, asum, sizeof(a), hipMemcpyDeviceToHost, s));
    SBX_HIP(hipMemcpyAsync(b4, D.bulk, sizeof(b4), hipMemcpyDeviceToHost, s));
    SBX_HIP(hipMemcpyAsync(z.data(), zsum, sizeof(double) * qy->n_z, hipMemcpyDeviceToHost, s));
    if (bin_r) SBX_HIP(hipMemcpyAsync(bin_r, br, sizeof(double) * nbins, hipMemcpyDeviceToHost, s));
    if (bin_vc) SBX_HIP(hipMemcpyAsync(bin_vc, bv, sizeof(double) * nbins, hipMemcpyDeviceToHost, s));
    if (bin_rms_z) SBX_HIP(hipMemcpyAsync(bin_rms_z, bz, sizeof(double) * nbins, hipMemcpyDeviceToHost, s));
    SBX_HIP(hipStreamSynchronize(s));
    res->e_heat = a[0];
    res->n_annulus = (int64_t)llround(a[1]);
    auto sd = [&](double s1, double s2) {
      if (a[1] <= 0) return 0.0;
      const double mu = s1 / a[1];
      return sqrt(std::max(s2 / a[1] - mu * mu, 0.0));
    };
    res->sig_R = sd(a[2], a[3]);
    res->sig_phi = sd(a[4], a[5]);
    res->sig_z = sd(a[6], a[7]);
    res->sig_tot2 = res->sig_R * res->sig_R + res->sig_phi * res->sig_phi + res->sig_z * res->sig_z;
    for (int k = 0; k < 3; ++k) res->bulk_v[k] = b4[1 + k] / b4[0];
    const double lo = qy->annulus[0], hi = qy->annulus[1];
    const double area = M_PI * (hi * hi - lo * lo), dz = 2.0 * qy->z_max / qy->n_z;
    if (rho_z)
      for (int k = 0; k < qy->n_z; ++k) rho_z[k] = z[k] / (area * dz);
    return SBX_OK;
  };
  const sbx_status rc = body();
  (void)hipStreamSynchronize(s);
  return rc;
}

// ------------------------------------------------------------ disc modes --
// first sorted position with R >= r (sorted radius keys)
__device__ __forceinline__ int64_t lower_bound_r(const uint64_t* key, int64_t n, double r) {
  const uint64_t kr = (uint64_t)__double_as_longlong(r);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < kr) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One block per annular bin [k dR, (k+1) dR): sum over its particles of
// M cos(m phi) and -M sin(m phi), m = 0..mmax, in a fixed order; divided by
// the bin area.  out[(k * (mmax + 1) + m) * 2 + {0, 1}] = re, im.
__global__ void __launch_bounds__(256)
    k_disc_modes(const uint64_t* __restrict__ key, const uint32_t* __restrict__ order, int64_t n,
                 const double* __restrict__ d3, const double* __restrict__ m1, double dR, int mmax,
                 double* __restrict__ out) {
  constexpr int kMaxM = 16;
  const int k = blockIdx.x;
  const int64_t s0 = lower_bound_r(key, n, k * dR), s1 = lower_bound_r(key, n, (k + 1) * dR);
  double a[2 * (kMaxM + 1)] = {};
  for (int64_t j = s0 + threadIdx.x; j < s1; j += 256) {
    const uint32_t i = order[j];
    const double ph = atan2(d3[3 * (size_t)i + 1], d3[3 * (size_t)i]);
    const double m = m1[i];
#pragma unroll
    for (int q = 0; q <= kMaxM; ++q) {
      if (q > mmax) break;
      double sn, cs;
      sincos((double)q * ph, &sn, &cs);
      a[2 * q] += m * cs;
      a[2 * q + 1] -= m * sn;
    }
  }
  __shared__ double res[2 * (kMaxM + 1)];
  block_rows<2 * (kMaxM + 1)>(a, res);
  __syncthreads();
  const double S = M_PI * dR * dR * ((double)(k + 1) * (k + 1) - (double)k * k);
  for (int q = threadIdx.x; q < 2 * (mmax + 1); q += 256) out[(size_t)k * 2 * (mmax + 1) + q] = res[q] / S;
}

template <typename T>
sbx_status modes_t(sbx_ctx* c, int comp, int galaxy, int nr, double rmax, int mmax, double* coeff) {
  hipStream_t s = c->stream;
  Disc D;
  auto body = [&]() -> sbx_status {
    SBX_TRY(disc_prepare<T>(c, comp, galaxy, D));
    double* out = nullptr;
    const size_t cnt = (size_t)nr * (mmax + 1) * 2;
    SBX_TRY(D.alloc((void**)&out, sizeof(double) * cnt));
    hipLaunchKernelGGL(k_disc_modes, dim3(nr), dim3(256), 0, s, D.key, D.order, D.n, D.d3, D.m1, rmax / nr,
                       mmax, out);
    SBX_HIP(hipGetLastError());
    SBX_HIP(hipMemcpyAsync(coeff, out, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
    SBX_HIP(hipStreamSynchronize(s));
    return SBX_OK;
  };
  const sbx_status rc = body();
  (void)hipStreamSynchronize(s);
  return rc;
}

}  // namespace

extern "C" {

sbx_status sbx_disc_analysis(sbx_ctx* c, const sbx_disc_query* q, sbx_disc_result* res,
                             double* bin_r, double* bin_vc, double* bin_rms_z, double* rho_z) {
  if (!c || !q || !res) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  if (c->batch && c->batch->pending) {
    set_error("the context's batch has queued work: call sbx_batch_sync first");
    return SBX_ESTATE;
  }
  if (!c->built || c->n == 0) {
    set_error("build_grids and load_particles first");
    return SBX_ESTATE;
  }
  if (q->n_bins < 1 || q->n_bins > kMaxBins || q->n_z < 1 || q->n_z > kMaxZ ||
      !(q->z_max > 0.0) || !(q->annulus[1] > q->annulus[0]) || !(q->annulus[0] >= 0.0) ||
      q->comp < 0 || q->comp >= kNComp || q->galaxy < 0 || q->galaxy >= c->ngal) {
    set_error("bad disc query (1 <= n_bins <= 2048, 1 <= n_z <= 1024, z_max > 0, "
              "0 <= R_lo < R_hi, component and galaxy in range)");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(c->cfg.device));
  std::memset(res, 0, sizeof(*res));
  return c->cfg.prec == SBX_FP64 ? disc_t<double>(c, q, res, bin_r, bin_vc, bin_rms_z, rho_z)
                                 : disc_t<float>(c, q, res, bin_r, bin_vc, bin_rms_z, rho_z);
}

sbx_status sbx_disc_modes(sbx_ctx* c, int32_t comp, int32_t galaxy, int32_t n_rbins, double r_max,
                          int32_t m_max, double* coeff) {
  if (!c || !coeff) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  if (c->batch && c->batch->pending) {
    set_error("the context's batch has queued work: call sbx_batch_sync first");
    return SBX_ESTATE;
  }
  if (!c->built || c->n == 0) {
    set_error("build_grids and load_particles first");
    return SBX_ESTATE;
  }
  if (n_rbins < 1 || n_rbins > 65536 || !(r_max > 0.0) || m_max < 0 || m_max > 16 || comp < 0 ||
      comp >= kNComp || galaxy < 0 || galaxy >= c->ngal) {
    set_error("bad mode query (1 <= n_rbins <= 65536, r_max > 0, 0 <= m_max <= 16)");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(c->cfg.device));
  return c->cfg.prec == SBX_FP64 ? modes_t<double>(c, comp, galaxy, n_rbins, r_max, m_max, coeff)
                                 : modes_t<float>(c, comp, galaxy, n_rbins, r_max, m_max, coeff);
}

}  // extern "C"
