// C ABI of the standalone isolated Poisson solves (Eqs. 1-5).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "ctx.h"

using namespace sbx;

// ------------------------------------------------------- no-alloc solves ---
// Work space of sbx_poisson_solve_noalloc: a fixed array in device memory of
// every GPU the library runs on, held until the process ends.  Layout per
// call: kPasses work counters, the solve descriptors, then per solve the X
// half spectrum and the C/D work arrays.  In host code the array's name is
// not a device address: kernels get the address from hipGetSymbolAddress,
// taken once per device when the first plan on that device is created.
constexpr size_t kNoallocBytes = 96ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDev = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDev] = {};
std::string g_scratch_err[kMaxDev];

// The device address of `scratch` on the current device (set-up, once per
// device; the failure message is kept for the entry point to report).
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDev) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    g_scratch_err[device] = std::string("hipGetSymbolAddress of the no-alloc work space failed: ") +
                            hipGetErrorString(e);
    return;
  }
  g_scratch[device] = ptr;
}

void* scratch_of(int device, std::string& why) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (device < 0 || device >= kMaxDev) {
    why = "device ordinal beyond the no-alloc work space table";
    return nullptr;
  }
  if (!g_scratch[device]) why = g_scratch_err[device].empty() ? "no-alloc work space not set up"
                                                               : g_scratch_err[device];
  return g_scratch[device];
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// One block: clear the work counters and write the descriptors of `batch`
// solves whose grids, work arrays and table are at the given places.
template <typename T>
__global__ void k_noalloc_setup(SolveDesc<T>* __restrict__ d, int batch, const T* rho, T* phi,
                                C2<T>* X, C2<T>* CD, const T* H, int N, size_t cells, size_t xe,
                                size_t ce, int* __restrict__ counters, int ncnt) {
  for (int i = threadIdx.x; i < ncnt; i += blockDim.x) counters[i] = 0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    SolveDesc<T> s;
    s.rho = rho + cells * b;
    s.rho2 = nullptr;
    s.phi = phi + cells * b;
    s.X = X + xe * b;
    s.C = CD + 2 * ce * b;
    s.D = s.C + ce;
    s.H = H;
    s.N = N;
    d[b] = s;
  }
}

}  // namespace

// Solve plans of a Poisson object are cached per (rho, phi, batch) so that a
// loop over the same buffers reuses its device tables.
struct PoissonPlan {
  const void* rho;
  void* phi;
  int batch;
  SolvePlan<float> p32;
  SolvePlan<double> p64;
};

struct sbx_poisson {
  int N = 0, prec = 0, device = 0;
  sbx_level geo;
  double G = 1.0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* H = nullptr;
  void* X = nullptr;
  void* C = nullptr;
  int cap = 0;
  double rel_imag = 0.0;
  int64_t bytes = 0;
  std::vector<PoissonPlan*> plans;
};


namespace {

constexpr int kMaxSolves = 40;

bool is_pow2_grid(int n) { return n >= 8 && n <= 256 && (n & (n - 1)) == 0; }  // solves per Poisson plan launch

template <typename T>
SolvePlan<T>& plan_of(PoissonPlan* q) {
  if constexpr (sizeof(T) == 8) return q->p64;
  else return q->p32;
}

template <typename T>
sbx_status poisson_solve_t(sbx_poisson* p, int batch, const void* rho, void* phi) {
  const size_t cells = (size_t)p->N * p->N * p->N;
  const int cap = std::min(batch, kMaxSolves);
  if (cap > p->cap) {
    SBX_HIP(hipStreamSynchronize(p->stream));
    for (auto* q : p->plans) {
      plan_destroy(q->p32);
      plan_destroy(q->p64);
      delete q;
    }
    p->plans.clear();
    free_ptr(p->X);
    free_ptr(p->C);
    p->cap = 0;
    SBX_TRY(dev_alloc(&p->X, x_elems(p->N) * sizeof(C2<T>) * cap));
    SBX_TRY(dev_alloc(&p->C, cd_elems(p->N) * sizeof(C2<T>) * cap));
    p->cap = cap;
    p->bytes = (int64_t)(h_elems(p->N) * sizeof(T) +
                         (x_elems(p->N) + cd_elems(p->N)) * sizeof(C2<T>) * cap);
  }
  for (int b0 = 0; b0 < batch; b0 += p->cap) {
    const int nb = std::min(p->cap, batch - b0);
    const void* r = (const T*)rho + cells * b0;
    void* f = (T*)phi + cells * b0;
    PoissonPlan* hit = nullptr;
    for (auto* q : p->plans)
      if (q->rho == r && q->phi == f && q->batch == nb) hit = q;
    if (!hit) {
      auto descs = [&](const T* rr, T* ff) {
        std::vector<SolveDesc<T>> d(nb);
        for (int i = 0; i < nb; ++i) {
          d[i].rho = rr + cells * i;
          d[i].rho2 = nullptr;
          d[i].phi = ff + cells * i;
          d[i].X = (C2<T>*)p->X + x_elems(p->N) * i;
          d[i].C = (C2<T>*)p->C + cd_elems(p->N) * i;
          d[i].D = d[i].C + c_elems(p->N);
          d[i].H = (const T*)p->H;
          d[i].N = p->N;
        }
        return d;
      };
      if (!tuning_cached((int)sizeof(T), std::vector<int>(nb, p->N))) {
        // tune on scratch grids, never on the caller's buffers
        T* scratch = nullptr;
        SBX_TRY(dev_alloc((void**)&scratch, sizeof(T) * cells * nb));
        SolvePlan<T> tmp;
        auto d = descs(scratch, scratch);
        const sbx_status rc = plan_create<T>(tmp, d.data(), nb, p->stream);
        plan_destroy(tmp);
        (void)hipFree(scratch);
        SBX_TRY(rc);
      }
      if (p->plans.size() >= 8) {
        SBX_HIP(hipStreamSynchronize(p->stream));
        plan_destroy(p->plans.front()->p32);
        plan_destroy(p->plans.front()->p64);
        delete p->plans.front();
        p->plans.erase(p->plans.begin());
      }
      hit = new PoissonPlan{r, f, nb, {}, {}};
      p->plans.push_back(hit);
      auto d = descs((const T*)r, (T*)f);
      SBX_TRY(plan_create<T>(plan_of<T>(hit), d.data(), nb, p->stream));
    }
    SBX_TRY(plan_run<T>(plan_of<T>(hit), p->stream));
  }
  return SBX_OK;
}

}  // namespace

extern "C" {

sbx_status sbx_poisson_create(int32_t n, double R, double q, double G, int32_t h0_mode, int32_t prec,
                              int32_t device, void* stream, sbx_poisson** out) {
  if (!out || !is_pow2_grid(n) || !(R > 0.0) || !(q > 0.0) || !(q <= 1.0) || !(G > 0.0) ||
      h0_mode < 0 || h0_mode > 2 || (prec != SBX_FP32 && prec != SBX_FP64)) {
    set_error("bad Poisson plan arguments");
    return SBX_EINVAL;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    set_error("no HIP device available");
    return SBX_EDEVICE;
  }
  SBX_TRY(set_device(device));
  sbx_poisson* p = new (std::nothrow) sbx_poisson();
  if (!p) return SBX_ENOMEM;
  p->N = n;
  p->prec = prec;
  p->device = device;
  p->geo = sbx_level{n, R, q};
  p->G = G;
  if (stream) {
    p->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&p->stream) != hipSuccess) {
      delete p;
      set_error("hipStreamCreate failed");
      return SBX_EDEVICE;
    }
    p->own_stream = true;
  }
  const size_t es = prec == SBX_FP64 ? 8 : 4;
  sbx_status rc = dev_alloc(&p->H, h_elems(n) * es);
  if (rc == SBX_OK) {
    const LevelDev L = make_level(p->geo);
    rc = prec == SBX_FP64 ? build_green<double>(n, L.l, L.lz, G, h0_mode, (double*)p->H, &p->rel_imag, p->stream)
                          : build_green<float>(n, L.l, L.lz, G, h0_mode, (float*)p->H, &p->rel_imag, p->stream);
  }
  // what sbx_poisson_solve_noalloc needs on this device, made here: the
  // work space address and the twiddle table of the plan's precision
  if (rc == SBX_OK) {
    scratch_setup(device);
    rc = prec == SBX_FP64 ? prepare_twiddles<double>(n, p->stream) : prepare_twiddles<float>(n, p->stream);
  }
  if (rc != SBX_OK) {
    sbx_poisson_destroy(p);
    return rc;
  }
  p->bytes = (int64_t)(h_elems(n) * es);
  *out = p;
  return SBX_OK;
}

void sbx_poisson_destroy(sbx_poisson* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (auto* q : p->plans) {
    plan_destroy(q->p32);
    plan_destroy(q->p64);
    delete q;
  }
  p->plans.clear();
  free_ptr(p->H);
  free_ptr(p->X);
  free_ptr(p->C);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

sbx_status sbx_poisson_solve(sbx_poisson* p, int32_t batch, const void* rho, void* phi) {
  if (!p || !rho || !phi || batch <= 0 || batch > 64) {
    set_error("bad Poisson solve arguments");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(p->device));
  return p->prec == SBX_FP64 ? poisson_solve_t<double>(p, batch, rho, phi)
                             : poisson_solve_t<float>(p, batch, rho, phi);
}

}  // extern "C"

namespace {

template <typename T>
sbx_status poisson_noalloc_t(sbx_poisson* p, int batch, const void* rho, void* phi, void* base) {
  const int N = p->N;
  const size_t cells = (size_t)N * N * N, xe = x_elems(N), ce = c_elems(N);
  const size_t off_desc = round256(sizeof(int) * kPasses);
  const size_t off_x = off_desc + round256(sizeof(SolveDesc<T>) * batch);
  const size_t off_cd = off_x + round256(sizeof(C2<T>) * xe * batch);
  const size_t need = off_cd + sizeof(C2<T>) * 2 * ce * batch;
  if (need > kNoallocBytes) {
    set_error("no-alloc solve of " + std::to_string(batch) + " grid(s) of " + std::to_string(N) +
              "^3 needs " + std::to_string(need) + " bytes of work space; the fixed no-alloc work "
              "space holds " + std::to_string(kNoallocBytes) + " (use sbx_poisson_solve)");
    return SBX_EINVAL;
  }
  unsigned char* s = (unsigned char*)base;
  int* counters = (int*)s;
  SolveDesc<T>* d = (SolveDesc<T>*)(s + off_desc);
  hipLaunchKernelGGL((k_noalloc_setup<T>), dim3(1), dim3(64), 0, p->stream, d, batch, (const T*)rho,
                     (T*)phi, (C2<T>*)(s + off_x), (C2<T>*)(s + off_cd), (const T*)p->H, N, cells, xe,
                     ce, counters, kPasses);
  SBX_HIP(hipGetLastError());
  return run_solves_noalloc<T>(d, batch, N, counters, p->stream);
}

}  // namespace

extern "C" {

sbx_status sbx_poisson_solve_noalloc(sbx_poisson* p, int32_t batch, const void* rho, void* phi) {
  if (!p || !rho || !phi || batch <= 0 || batch > 64) {
    set_error("bad Poisson solve arguments");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(p->device));
  std::string why;
  void* base = scratch_of(p->device, why);
  if (!base) {
    set_error(why);
    return SBX_EDEVICE;
  }
  return p->prec == SBX_FP64 ? poisson_noalloc_t<double>(p, batch, rho, phi, base)
                             : poisson_noalloc_t<float>(p, batch, rho, phi, base);
}

sbx_status sbx_poisson_green(sbx_poisson* p, double* out, double* rel_imag) {
  if (!p || !out) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(p->device));
  const size_t n = h_elems(p->N);
  double* stage = nullptr;
  SBX_TRY(dev_alloc((void**)&stage, n * sizeof(double)));
  sbx_status rc = p->prec == SBX_FP64 ? launch_convert_out<double>((double*)p->H, stage, n, p->stream)
                                      : launch_convert_out<float>((float*)p->H, stage, n, p->stream);
  if (rc == SBX_OK) {
    if (hipMemcpyAsync(out, stage, n * sizeof(double), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess) {
      set_error("copy of the Green's table failed");
      rc = SBX_EDEVICE;
    }
  }
  (void)hipFree(stage);
  if (rel_imag) *rel_imag = p->rel_imag;
  return rc;
}

int64_t sbx_poisson_bytes(sbx_poisson* p) { return p ? p->bytes : 0; }

sbx_status sbx_set_fft_schedule(int32_t v) { return set_fft_schedule((int)v); }

sbx_status sbx_set_fft_form(int32_t f) { return set_fft_form((int)f); }

sbx_status sbx_set_plane_threads(int32_t nt) { return set_plane_threads((int)nt); }

int64_t sbx_fft_tuning_report(char* out, int64_t cap) {
  const std::string r = tuning_report();
  if (out && cap > 0) {
    const size_t n = std::min((size_t)(cap - 1), r.size());
    std::memcpy(out, r.data(), n);
    out[n] = 0;
  }
  return (int64_t)r.size();
}

}  // extern "C"
