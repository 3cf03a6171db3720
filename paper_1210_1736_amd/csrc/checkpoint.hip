// Checkpoint files of a context: the paper's runs evolve a model, keep it
// and reuse it (Sec. 3.1 and 4.1: galaxy and satellite are relaxed in
// isolation, then combined), so a state is written and read back whole.
//
// Format (little-endian, fields written one by one, no padding):
//   "SBXCKPT1", int32 version (2), int32 prec, double G, int32 h0_mode,
//   int32 taylor, int32 ngal, int32 merge5, int32 sort_every,
//   int32 fixed-point mass assignment (version 2 only), int32 solved,
//   int64 n, int64 step_count, double dt, per galaxy: int32 n_levels,
//   int32 centring, 3 x (int32 n, double R, double q), double centre[3],
//   double outer_centre[3]; then double centres[3 * ngal] (the centres of
//   the last solve), then per particle in the caller's order: x[3 n],
//   v[3 n] (staggered), m[n] as doubles, comp[n], gal[n], lost[n] as bytes,
//   and the closing tag "SBXEND01".
#include <cstdio>

#include "ctx.h"

using namespace sbx;

namespace {

constexpr char kMagic[8] = {'S', 'B', 'X', 'C', 'K', 'P', 'T', '1'};
constexpr char kTail[8] = {'S', 'B', 'X', 'E', 'N', 'D', '0', '1'};
constexpr int32_t kVersion = 2;  // version 1 files (no mass assignment flag) still load

struct Writer {
  FILE* f;
  bool ok = true;
  void raw(const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; }
  template <typename V>
  void put(V v) { raw(&v, sizeof(v)); }
};

struct Reader {
  std::vector<char> buf;
  size_t at = 0;
  bool ok = true;
  void raw(void* p, size_t n) {
    if (!ok || at + n > buf.size()) {
      ok = false;
      return;
    }
    std::memcpy(p, buf.data() + at, n);
    at += n;
  }
  template <typename V>
  V get() {
    V v{};
    raw(&v, sizeof(v));
    return v;
  }
};

// Masses, components and galaxies in the caller's order (host).
template <typename T>
sbx_status get_static_t(sbx_ctx* c, double* m, int8_t* comp, int8_t* gal) {
  const PSet& q = c->set[c->cur];
  const int64_t n = c->n;
  double* stage = nullptr;
  SBX_TRY(dev_alloc((void**)&stage, sizeof(double) * 2 * n));
  auto run = [&]() -> sbx_status {
    SBX_TRY(launch_convert_out<T>((const T*)q.m, stage, n, c->stream));
    SBX_TRY(launch_unpermute<double>(stage, q.id, stage + n, n, 1, c->stream));
    SBX_HIP(hipMemcpyAsync(m, stage + n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    int8_t* b = (int8_t*)stage;
    SBX_TRY(launch_unpermute<int8_t>(q.comp, q.id, b, n, 1, c->stream));
    SBX_HIP(hipMemcpyAsync(comp, b, n, hipMemcpyDeviceToHost, c->stream));
    SBX_HIP(hipStreamSynchronize(c->stream));
    SBX_TRY(launch_unpermute<int8_t>(q.gal, q.id, b, n, 1, c->stream));
    SBX_HIP(hipMemcpyAsync(gal, b, n, hipMemcpyDeviceToHost, c->stream));
    SBX_HIP(hipStreamSynchronize(c->stream));
    return SBX_OK;
  };
  const sbx_status rc = run();
  (void)hipFree(stage);
  return rc;
}

}  // namespace

extern "C" {

sbx_status sbx_save(sbx_ctx* c, const char* path) {
  if (!c || !path) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  if (c->batch && c->batch->pending) {
    set_error("the context's batch has queued work: call sbx_batch_sync first");
    return SBX_ESTATE;
  }
  if (!c->built || c->n == 0) {
    set_error("nothing to save: build_grids and load particles first");
    return SBX_ESTATE;
  }
  SBX_TRY(set_device(c->cfg.device));
  const int64_t n = c->n;
  std::vector<double> x(3 * n), v(3 * n), m(n), cen(3 * c->ngal);
  std::vector<int8_t> comp(n), gal(n);
  std::vector<uint8_t> lost(n);
  SBX_TRY(get_impl(c, x.data(), v.data(), lost.data(), false));
  SBX_TRY(c->cfg.prec == SBX_FP64 ? get_static_t<double>(c, m.data(), comp.data(), gal.data())
                                  : get_static_t<float>(c, m.data(), comp.data(), gal.data()));
  SBX_TRY(sbx_get_centres(c, cen.data()));
  FILE* f = std::fopen(path, "wb");
  if (!f) {
    set_error(std::string("cannot open ") + path + " for writing");
    return SBX_EINVAL;
  }
  Writer w{f};
  w.raw(kMagic, 8);
  w.put<int32_t>(kVersion);
  w.put<int32_t>(c->cfg.prec);
  w.put<double>(c->cfg.G);
  w.put<int32_t>(c->cfg.h0_mode);
  w.put<int32_t>(c->cfg.taylor);
  w.put<int32_t>(c->ngal);
  w.put<int32_t>(c->sys.merge5);
  w.put<int32_t>(c->sort_every);
  w.put<int32_t>(c->fix_on ? 1 : 0);
  w.put<int32_t>(c->solved ? 1 : 0);
  w.put<int64_t>(n);
  w.put<int64_t>(c->step_count);
  w.put<double>(c->dt_dev);
  for (int g = 0; g < c->ngal; ++g) {
    const sbx_hierarchy& h = c->hh[g];
    w.put<int32_t>(h.n_levels);
    w.put<int32_t>(h.centring);
    for (int k = 0; k < 3; ++k) {
      w.put<int32_t>(h.lv[k].n);
      w.put<double>(h.lv[k].R);
      w.put<double>(h.lv[k].q);
    }
    for (int k = 0; k < 3; ++k) w.put<double>(h.centre[k]);
    for (int k = 0; k < 3; ++k) w.put<double>(h.outer_centre[k]);
  }
  w.raw(cen.data(), sizeof(double) * cen.size());
  w.raw(x.data(), sizeof(double) * x.size());
  w.raw(v.data(), sizeof(double) * v.size());
  w.raw(m.data(), sizeof(double) * m.size());
  w.raw(comp.data(), n);
  w.raw(gal.data(), n);
  w.raw(lost.data(), n);
  w.raw(kTail, 8);
  const bool closed = std::fclose(f) == 0;
  if (!w.ok || !closed) {
    set_error(std::string("write error on ") + path);
    return SBX_EINVAL;
  }
  return SBX_OK;
}

sbx_status sbx_load(sbx_ctx* c, const char* path) {
  if (!c || !path) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return SBX_EINVAL;
  }
  Reader r;
  char chunk[1 << 16];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) r.buf.insert(r.buf.end(), chunk, chunk + got);
  std::fclose(f);
  char magic[8];
  r.raw(magic, 8);
  const int32_t version = r.ok ? r.get<int32_t>() : 0;
  if (!r.ok || std::memcmp(magic, kMagic, 8) != 0 || version < 1 || version > kVersion) {
    set_error(std::string(path) + " is not a checkpoint of this library (versions 1 and 2)");
    return SBX_EINVAL;
  }
  const int32_t prec = r.get<int32_t>();
  const double G = r.get<double>();
  const int32_t h0 = r.get<int32_t>(), taylor = r.get<int32_t>(), ngal = r.get<int32_t>();
  const int32_t merge5 = r.get<int32_t>(), sort_every = r.get<int32_t>();
  const int32_t fixed = version >= 2 ? r.get<int32_t>() : 0;
  const int32_t solved = r.get<int32_t>();
  const int64_t n = r.get<int64_t>(), steps = r.get<int64_t>();
  const double dt = r.get<double>();
  if (!r.ok || ngal < 1 || ngal > kMaxGal || n <= 0 || n >= ((int64_t)1 << 31) || sort_every < 0 ||
      (merge5 != 0 && merge5 != 1) || (fixed != 0 && fixed != 1)) {
    set_error(std::string(path) + ": corrupt header");
    return SBX_EINVAL;
  }
  if (prec != c->cfg.prec || G != c->cfg.G || h0 != c->cfg.h0_mode ||
      (taylor != 0) != (c->cfg.taylor != 0)) {
    set_error(std::string(path) + " was written by a context of another precision, G, h0_mode or "
              "taylor setting");
    return SBX_EINVAL;
  }
  std::vector<sbx_hierarchy> hh(ngal);
  for (auto& h : hh) {
    std::memset(&h, 0, sizeof(h));
    h.n_levels = r.get<int32_t>();
    h.centring = r.get<int32_t>();
    for (int k = 0; k < 3; ++k) {
      h.lv[k].n = r.get<int32_t>();
      h.lv[k].R = r.get<double>();
      h.lv[k].q = r.get<double>();
    }
    for (int k = 0; k < 3; ++k) h.centre[k] = r.get<double>();
    for (int k = 0; k < 3; ++k) h.outer_centre[k] = r.get<double>();
  }
  std::vector<double> cen(3 * ngal), x(3 * n), v(3 * n), m(n);
  std::vector<int8_t> comp(n), gal(n);
  std::vector<uint8_t> lost(n);
  r.raw(cen.data(), sizeof(double) * cen.size());
  r.raw(x.data(), sizeof(double) * x.size());
  r.raw(v.data(), sizeof(double) * v.size());
  r.raw(m.data(), sizeof(double) * m.size());
  r.raw(comp.data(), n);
  r.raw(gal.data(), n);
  r.raw(lost.data(), n);
  char tail[8];
  r.raw(tail, 8);
  if (!r.ok || std::memcmp(tail, kTail, 8) != 0 || r.at != r.buf.size()) {
    set_error(std::string(path) + ": truncated or corrupt checkpoint");
    return SBX_EINVAL;
  }
  SBX_TRY(sbx_set_outer_merge(c, merge5));
  SBX_TRY(sbx_set_deterministic_deposit(c, fixed));
  SBX_TRY(sbx_build_grids(c, ngal, hh.data()));
  SBX_TRY(load_impl(c, n, x.data(), v.data(), m.data(), comp.data(), gal.data(), false));
  // load_impl leaves the caller's order (cur = 0): the flags go straight in
  SBX_HIP(hipMemcpy(c->set[c->cur].lost, lost.data(), n, hipMemcpyHostToDevice));
  c->sort_every = sort_every;
  c->step_count = steps;
  c->dt_dev = dt;
  c->solved = solved != 0;
  if (c->solved)
    SBX_HIP(hipMemcpy(c->centres, cen.data(), sizeof(double) * cen.size(), hipMemcpyHostToDevice));
  return upload_inst(c);
}

}  // extern "C"
