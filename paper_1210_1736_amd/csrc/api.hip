// C ABI of the library: contexts (particles, grids, forces, steps).  Host
// code only orchestrates: every step of the method runs in the kernels of
// fft.hip and particles.hip.
#include "ctx.h"

namespace sbx {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

static bool is_pow2_grid(int n) { return n >= 8 && n <= 256 && (n & (n - 1)) == 0; }

// Geometry of one level as the method reads it: the usable N-4 cells span
// 2R, so l = 2R/(N-4); the z cell length of a flattened grid is q*l.
LevelDev make_level(const sbx_level& s) {
  LevelDev L;
  L.N = s.n;
  L.half = (double)s.n / 2.0;
  L.l = (2.0 * s.R) / (double)(s.n - 4);
  L.lz = s.q * L.l;
  L.gx = 1.0 / L.l;
  L.gz = 1.0 / L.lz;
  L.inv_q = 1.0 / s.q;
  L.R2 = s.R * s.R;
  L.c_2l = 0.5 / L.l;
  L.c_2lz = 0.5 / L.lz;
  L.c_l2 = 1.0 / (L.l * L.l);
  L.c_lz2 = 1.0 / (L.lz * L.lz);
  L.c_4ll = 1.0 / (4.0 * L.l * L.l);
  L.c_4llz = 1.0 / (4.0 * L.l * L.lz);
  return L;
}

double q_crit_of(int n, double Rc, double Ro, double Rs) {
  const double a = Rc / Ro;
  const double b = 4.0 / (n - 4) * Rs / Ro;
  return a > b ? a : b;
}

bool same_level(const sbx_level& a, const sbx_level& b) {
  return a.n == b.n && a.R == b.R && a.q == b.q;
}

sbx_status validate(int ng, const sbx_hierarchy* h) {
  if (!h || ng < 1 || ng > kMaxGal) {
    set_error("1 to 8 galaxies required");
    return SBX_EINVAL;
  }
  const int N0 = h[0].lv[0].n;
  for (int g = 0; g < ng; ++g) {
    const sbx_hierarchy& hh = h[g];
    if (hh.n_levels != 1 && hh.n_levels != 3) {
      set_error("a hierarchy has 1 or 3 levels");
      return SBX_EINVAL;
    }
    if (hh.centring != SBX_CENTRE_FIXED && hh.centring != SBX_CENTRE_COM &&
        hh.centring != SBX_CENTRE_DENSITY) {
      set_error("unknown centring");
      return SBX_EINVAL;
    }
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(hh.centre[k]) || !std::isfinite(hh.outer_centre[k])) {
        set_error("centres must be finite");
        return SBX_EINVAL;
      }
    for (int k = 0; k < hh.n_levels; ++k) {
      const sbx_level& L = hh.lv[k];
      if (!is_pow2_grid(L.n)) {
        set_error("grid size must be a power of two in 8..256");
        return SBX_EINVAL;
      }
      if (L.n != N0) {
        set_error("all grids have the same number of cells (Sec. 2.1)");
        return SBX_EINVAL;
      }
      if (!(L.R > 0.0) || !std::isfinite(L.R) || !(L.q > 0.0) || !(L.q <= 1.0)) {
        set_error("need R > 0 and 0 < q <= 1");
        return SBX_EINVAL;
      }
    }
    if (hh.n_levels == 1) {
      if (ng != 1 || hh.centring != SBX_CENTRE_FIXED) {
        set_error("a single grid is the fixed global grid of one galaxy");
        return SBX_EINVAL;
      }
      continue;
    }
    const sbx_level &L1 = hh.lv[0], &L2 = hh.lv[1], &L3 = hh.lv[2];
    if (!(L1.R < L2.R && L2.R < L3.R)) {
      set_error("levels must nest: R1 < R2 < R3");
      return SBX_EINVAL;
    }
    if (L3.q != 1.0) {
      set_error("the global grid is not flattened");
      return SBX_EINVAL;
    }
    if (g > 0 && (L1.q != 1.0 || L2.q != 1.0)) {
      set_error("q < 1 applies only to the first galaxy (Sec. 2.2.2)");
      return SBX_EINVAL;
    }
    const double qc = q_crit_of(L2.n, L1.R, L2.R, L3.R);
    if (L2.q < qc) {
      set_error("flattening q = " + std::to_string(L2.q) + " below q_crit = " +
                std::to_string(qc) + " (Eq. 9)");
      return SBX_EQCRIT;
    }
    if (L2.q * L2.R < L1.q * L1.R) {
      set_error("flattened middle grid must still cover the inner grid");
      return SBX_EINVAL;
    }
    if (g > 0) {
      const sbx_hierarchy& h0 = h[0];
      if (!same_level(L3, h0.lv[2]) || std::memcmp(hh.outer_centre, h0.outer_centre,
                                                   sizeof(hh.outer_centre)) != 0) {
        set_error("several galaxies share one global grid");
        return SBX_EINVAL;
      }
    }
  }
  return SBX_OK;
}

sbx_status dev_alloc(void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("out of device memory (" + std::to_string(bytes) + " bytes)");
    return SBX_ENOMEM;
  }
  return SBX_OK;
}

void free_ptr(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

sbx_status set_device(int dev) {
  SBX_HIP(hipSetDevice(dev));
  return SBX_OK;
}

void to_diag(const double* r, sbx_diag* d) {
  std::memset(d, 0, sizeof(*d));
  for (int c = 0; c < kNComp; ++c) {
    d->ekin[c] = r[kDiagComp * c + 0];
    d->epot[c] = r[kDiagComp * c + 1];
    d->L[c][0] = r[kDiagComp * c + 2];
    d->L[c][1] = r[kDiagComp * c + 3];
    d->L[c][2] = r[kDiagComp * c + 4];
    d->n_live[c] = (int64_t)llround(r[kDiagComp * c + 5]);
  }
  const double* q = r + kDiagDisc;
  if (q[4] > 0) {
    const double mR = q[0] / q[4], mz = q[2] / q[4];
    d->disc_sigR = std::sqrt(std::fmax(q[1] / q[4] - mR * mR, 0.0));
    d->disc_sigz = std::sqrt(std::fmax(q[3] / q[4] - mz * mz, 0.0));
  }
  d->n_lost = (int64_t)llround(r[kDiagLost]);
}

template <typename T>
static PartDev<T> pset_dev(const PSet& s, int64_t n) {
  PartDev<T> p;
  for (int k = 0; k < 3; ++k) {
    p.x[k] = (T*)s.x[k];
    p.v[k] = (T*)s.v[k];
  }
  p.m = (T*)s.m;
  p.comp = s.comp;
  p.gal = s.gal;
  p.lost = s.lost;
  p.id = s.id;
  p.n = n;
  return p;
}

template <typename T>
InstDev<T> inst_of(const sbx_ctx* c) {
  InstDev<T> I;
  std::memset(&I, 0, sizeof(I));
  I.p[0] = pset_dev<T>(c->set[0], c->n);
  I.p[1] = pset_dev<T>(c->set[1], c->n);
  I.sys = c->sys;
  for (int g = 0; g < kMaxGal; ++g)
    for (int k = 0; k < kSlots; ++k) I.G.g[g][k] = (T*)c->grid[g][k];
  I.centres = c->centres;
  I.com_partial = c->com_partial;
  I.pre_partial = c->pre_partial;
  I.diag_partial = c->diag_partial;
  I.diag_out = c->diag_one;
  I.acc = c->acc;
  I.pot = c->pot;
  I.grid_block = (T*)c->grid_block;
  I.grid_elems = c->mass_elems;
  I.key = c->key;
  I.rank = c->rank;
  I.count = c->count;
  I.part_base = 0;
  I.dm_hist = c->dm_hist;
  I.dm_elems = c->dm_elems;
  I.dm_aux = c->dm_aux;
  I.dm_partial = c->dm_partial;
  I.dm_mmax = c->dm_mmax;
  I.dt = c->dt_dev;
  I.n = c->n;
  I.fix = c->fix;
  return I;
}

template InstDev<float> inst_of<float>(const sbx_ctx*);
template InstDev<double> inst_of<double>(const sbx_ctx*);

sbx_status upload_inst(sbx_ctx* c) {
  SBX_HIP(hipStreamSynchronize(c->stream));
  if (c->built && !c->solved) {
    // the centres a solve starts from (density-maximum centring) until the
    // first solve has computed them
    double hc[3 * kMaxGal];
    for (int g = 0; g < c->ngal; ++g)
      for (int k = 0; k < 3; ++k) hc[3 * g + k] = c->hh[g].centre[k];
    SBX_HIP(hipMemcpy(c->centres, hc, sizeof(double) * 3 * c->ngal, hipMemcpyHostToDevice));
  }
  if (c->cfg.prec == SBX_FP64) {
    const InstDev<double> I = inst_of<double>(c);
    SBX_HIP(hipMemcpy(c->d_inst, &I, sizeof(I), hipMemcpyHostToDevice));
  } else {
    const InstDev<float> I = inst_of<float>(c);
    SBX_HIP(hipMemcpy(c->d_inst, &I, sizeof(I), hipMemcpyHostToDevice));
  }
  SBX_HIP(hipMemcpy(c->d_cur, &c->cur, sizeof(int), hipMemcpyHostToDevice));
  return SBX_OK;
}

}  // namespace sbx

using namespace sbx;

namespace {

template <typename P>
void free_typed(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void free_particles(sbx_ctx* c) {
  if (c->bound) {
    // borrowed storage stays with the caller; only the id array is ours
    free_typed(c->set[0].id);
    c->set[0] = PSet();
    c->bound = false;
  }
  for (int s = 0; s < 2; ++s) {
    PSet& q = c->set[s];
    for (int k = 0; k < 3; ++k) {
      free_ptr(q.x[k]);
      free_ptr(q.v[k]);
    }
    free_ptr(q.m);
    free_typed(q.comp);
    free_typed(q.gal);
    free_typed(q.lost);
    free_typed(q.id);
  }
  free_typed(c->key);
  free_typed(c->rank);
  free_typed(c->acc);
  free_typed(c->pot);
  free_ptr(c->adj_work);
  c->adj_work_bytes = 0;
  c->acc_n = 0;
  c->n = 0;
  c->cur = 0;
  c->com_fresh = false;
}

void free_grids(sbx_ctx* c) {
  plan_destroy(c->plan32);
  plan_destroy(c->plan64);
  plan_destroy(c->adj32);
  plan_destroy(c->adj64);
  free_ptr(c->adj_block);
  free_ptr(c->adj_work);
  c->adj_work_bytes = 0;
  free_ptr(c->grid_block);
  free_typed(c->fix);
  free_typed(c->count);
  free_typed(c->scan_tmp);
  free_typed(c->dm_hist);
  free_typed(c->dm_aux);
  free_typed(c->dm_partial);
  c->dm_elems = 0;
  c->bins = 0;
  for (auto& g : c->greens) free_ptr(g.H);
  c->greens.clear();
  free_ptr(c->X);
  free_ptr(c->C);
  std::memset(c->grid, 0, sizeof(c->grid));
  c->grid_elems = 0;
  c->mass_elems = 0;
  c->built = false;
  c->solved = false;
}

// grids allocated per galaxy (fields and mass-only), and the solved ones
int slot_count(const sbx_hierarchy& h) { return h.n_levels == 3 ? kSlots : 1; }
int field_slot_count(const sbx_hierarchy& h) { return h.n_levels == 3 ? kFieldSlots : 1; }
int slot_level_of(const sbx_hierarchy& h, int slot) {
  if (h.n_levels == 1) return 0;
  static const int lv[kSlots] = {0, 1, 1, 2, 2, 1, 2};
  return lv[slot];
}

template <typename T>
sbx_status build_grids_t(sbx_ctx* c) {
  const int N = c->N;
  const size_t cells = (size_t)N * N * N;
  int total = 0;
  for (int g = 0; g < c->ngal; ++g) total += c->nslots[g];
  c->nsolves = total;
  c->grid_elems = cells * total;
  SBX_TRY(dev_alloc(&c->grid_block, sizeof(T) * c->grid_elems));
  // the slots that receive masses first (they are cleared every step), then
  // the two that only ever hold fields of summed grids (2 and 4)
  int s = 0;
  for (int g = 0; g < c->ngal; ++g)
    for (int k = 0; k < c->nslots[g]; ++k)
      if (c->nslots[g] == 1 || (k != 2 && k != 4)) c->grid[g][k] = (T*)c->grid_block + cells * (s++);
  c->mass_elems = cells * s;
  for (int g = 0; g < c->ngal; ++g)
    if (c->nslots[g] > 1)
      for (int k : {2, 4}) c->grid[g][k] = (T*)c->grid_block + cells * (s++);
  if (c->fix_on) {
    SBX_TRY(dev_alloc((void**)&c->fix, sizeof(unsigned long long) * c->mass_elems));
    SBX_HIP(hipMemsetAsync(c->fix, 0, sizeof(unsigned long long) * c->mass_elems, c->stream));
  }
  // Green's tables, one per distinct level geometry
  for (int g = 0; g < c->ngal; ++g)
    for (int lv = 0; lv < c->hh[g].n_levels; ++lv) {
      const sbx_level& geo = c->hh[g].lv[lv];
      bool have = false;
      for (auto& e : c->greens) have = have || same_level(e.geo, geo);
      if (have) continue;
      Green e{geo, nullptr, 0.0};
      SBX_TRY(dev_alloc(&e.H, h_elems(N) * sizeof(T)));
      c->greens.push_back(e);
      const LevelDev L = make_level(geo);
      SBX_TRY(build_green<T>(N, L.l, L.lz, c->cfg.G, c->cfg.h0_mode, (T*)c->greens.back().H,
                             &c->greens.back().rel_imag, c->stream));
    }
  SBX_TRY(dev_alloc(&c->X, x_elems(N) * sizeof(C2<T>) * total));
  SBX_TRY(dev_alloc(&c->C, cd_elems(N) * sizeof(C2<T>) * total));
  // one persistent plan for all solves of a step
  std::vector<SolveDesc<T>> descs;
  int s2 = 0;
  for (int g = 0; g < c->ngal; ++g)
    for (int k = 0; k < field_slot_count(c->hh[g]); ++k, ++s2) {
      if (c->sys.merge5 && g > 0 && k == 3) continue;  // summed into galaxy 0's grid 5
      SolveDesc<T> d;
      d.rho = (const T*)c->grid[g][k];
      d.rho2 = nullptr;
      if (c->hh[g].n_levels == 3 && k == 2) {         // grids 2 + 3
        d.rho = (const T*)c->grid[g][kSlotG2];
        d.rho2 = (const T*)c->grid[g][1];
      } else if (c->hh[g].n_levels == 3 && k == 4) {  // grids 4 + 5 (4 alone if merged)
        d.rho = (const T*)c->grid[g][kSlotG4];
        d.rho2 = c->sys.merge5 ? nullptr : (const T*)c->grid[g][3];
      }
      d.phi = (T*)c->grid[g][k];
      d.X = (C2<T>*)c->X + x_elems(N) * s2;
      d.C = (C2<T>*)c->C + cd_elems(N) * s2;
      d.D = d.C + c_elems(N);
      d.H = nullptr;
      d.N = N;
      for (auto& e : c->greens)
        if (same_level(e.geo, c->hh[g].lv[c->slot_level[g][k]])) d.H = (const T*)e.H;
      descs.push_back(d);
    }
  c->nsolves = (int)descs.size();
  if constexpr (sizeof(T) == 8) SBX_TRY(plan_create<T>(c->plan64, descs.data(), (int)descs.size(), c->stream));
  else SBX_TRY(plan_create<T>(c->plan32, descs.data(), (int)descs.size(), c->stream));
  // counting-sort bins (the cells of every level of every galaxy)
  c->bins = sort_bins(c->sys);
  SBX_TRY(dev_alloc((void**)&c->count, sizeof(uint32_t) * (c->bins + 1)));
  SBX_TRY(dev_alloc((void**)&c->scan_tmp, sizeof(uint32_t) * scan_tmp_elems(c->bins + 1)));
  // density-maximum centring: one N^3 integer histogram per galaxy
  bool dm = false;
  for (int g = 0; g < c->ngal; ++g) dm = dm || c->hh[g].centring == SBX_CENTRE_DENSITY;
  if (dm) {
    c->dm_elems = cells * c->ngal;
    SBX_TRY(dev_alloc((void**)&c->dm_hist, sizeof(unsigned long long) * c->dm_elems));
    SBX_TRY(dev_alloc((void**)&c->dm_aux, sizeof(unsigned long long) * kDmAux));
    SBX_TRY(dev_alloc((void**)&c->dm_partial, sizeof(double) * (size_t)kRedBlocks * kPreVals));
  }
  return SBX_OK;
}

template <typename T>
const InstDev<T>* dinst(sbx_ctx* c) {
  return (const InstDev<T>*)c->d_inst;
}

// Loss test, centres, mass assignment and all isolated solves of one step.
template <typename T>
sbx_status field_solve_t(sbx_ctx* c) {
  const std::vector<InstInfo> info{info_of(c)};
  c->rec.mark(PH_START, c->stream);
  if (c->com_fresh && c->dm_elems == 0) {
    SBX_TRY(launch_zero_and_centres<T>(dinst<T>(c), info, c->stream));
  } else {
    SBX_TRY(launch_zero_grids<T>(dinst<T>(c), info, c->stream));
    c->rec.mark(PH_ZERO, c->stream);
    SBX_TRY(launch_centres<T>(dinst<T>(c), c->d_cur, info, c->com_fresh, c->stream));
  }
  c->rec.mark(PH_PRE, c->stream);
  SBX_TRY(launch_deposit<T>(dinst<T>(c), c->d_cur, info, c->stream));
  c->rec.mark(PH_DEPOSIT, c->stream);
  if constexpr (sizeof(T) == 8) SBX_TRY(plan_run<T>(c->plan64, c->stream, &c->rec));
  else SBX_TRY(plan_run<T>(c->plan32, c->stream, &c->rec));
  c->solved = true;
  c->grids_fields = true;
  return SBX_OK;
}

template <typename T>
sbx_status force_t(sbx_ctx* c, int mode) {
  const std::vector<InstInfo> info{info_of(c)};
  SBX_TRY(launch_force<T>(dinst<T>(c), c->d_cur, info, mode, c->stream));
  c->rec.mark(PH_FORCE, c->stream);
  if (mode & 1) c->com_fresh = true;
  return SBX_OK;
}

// Reorder the particles by the cell of their finest grid, at the centres of
// the last solve (or the current centre of mass before the first one).
template <typename T>
sbx_status sort_t(sbx_ctx* c) {
  const std::vector<InstInfo> info{info_of(c)};
  c->rec.mark(PH_START, c->stream);
  if (!c->solved) SBX_TRY(launch_centres<T>(dinst<T>(c), c->d_cur, info, false, c->stream, false));
  SBX_TRY(launch_sort<T>(dinst<T>(c), c->d_cur, info, c->count, c->bins + 1, c->scan_tmp, c->stream));
  c->cur ^= 1;
  c->rec.mark(PH_SORT, c->stream);
  return SBX_OK;
}

sbx_status field_solve(sbx_ctx* c) {
  return c->cfg.prec == SBX_FP64 ? field_solve_t<double>(c) : field_solve_t<float>(c);
}
sbx_status force(sbx_ctx* c, int mode) {
  return c->cfg.prec == SBX_FP64 ? force_t<double>(c, mode) : force_t<float>(c, mode);
}
sbx_status sort_particles(sbx_ctx* c) {
  return c->cfg.prec == SBX_FP64 ? sort_t<double>(c) : sort_t<float>(c);
}

void free_recorder(Recorder& r) {
  for (int i = 0; i < r.cap; ++i) (void)hipEventDestroy(r.ev[i]);
  delete[] r.ev;
  delete[] r.tag;
  r = Recorder();
}

sbx_status check_ready(sbx_ctx* c) {
  if (!c) {
    set_error("null context");
    return SBX_EINVAL;
  }
  if (c->batch && c->batch->pending) {
    set_error("the context's batch has queued work: call sbx_batch_sync first");
    return SBX_ESTATE;
  }
  if (!c->built) {
    set_error("build_grids has not been called");
    return SBX_ESTATE;
  }
  if (c->n == 0 || !c->set[0].x[0]) {
    set_error("no particles loaded");
    return SBX_ESTATE;
  }
  return set_device(c->cfg.device);
}

sbx_status ensure_acc(sbx_ctx* c) {
  if (c->acc_n == c->n && c->acc) return SBX_OK;
  free_typed(c->acc);
  free_typed(c->pot);
  SBX_TRY(dev_alloc((void**)&c->acc, sizeof(double) * 3 * c->n));
  SBX_TRY(dev_alloc((void**)&c->pot, sizeof(double) * c->n));
  c->acc_n = c->n;
  return upload_inst(c);
}

sbx_status set_dt(sbx_ctx* c, double dt) {
  if (c->dt_dev == dt) return SBX_OK;
  c->dt_dev = dt;
  return upload_inst(c);
}


// ------------------------------------------------------ segment adjoint ----
template <typename T>
GridsDev<T> adj_grids(sbx_ctx* c) {
  GridsDev<T> G;
  std::memset(&G, 0, sizeof(G));
  for (int g = 0; g < c->ngal; ++g)
    for (int k = 0; k < c->nslots[g]; ++k)
      G.g[g][k] = (T*)c->adj_block + ((T*)c->grid[g][k] - (T*)c->grid_block);
  return G;
}

template <typename T>
sbx_status ensure_adjoint(sbx_ctx* c) {
  if (c->adj_block) return SBX_OK;
  SBX_TRY(dev_alloc(&c->adj_block, sizeof(T) * c->grid_elems));
  SolvePlan<T>& fwd = sizeof(T) == 8 ? (SolvePlan<T>&)c->plan64 : (SolvePlan<T>&)c->plan32;
  std::vector<SolveDesc<T>> d = fwd.host;
  for (auto& e : d) {
    // the adjoint sources are scattered into the slots the fields are read from
    T* a = (T*)c->adj_block + ((const T*)e.phi - (const T*)c->grid_block);
    e.rho = a;
    e.rho2 = nullptr;
    e.phi = a;
  }
  SolvePlan<T>& adj = sizeof(T) == 8 ? (SolvePlan<T>&)c->adj64 : (SolvePlan<T>&)c->adj32;
  return plan_create<T>(adj, d.data(), (int)d.size(), c->stream);
}

template <typename T>
sbx_status copy_set(sbx_ctx* c, const PSet& dst, const PSet& src, bool with_v, bool with_lost) {
  const size_t b = sizeof(T) * c->n;
  for (int k = 0; k < 3; ++k) {
    SBX_HIP(hipMemcpyAsync(dst.x[k], src.x[k], b, hipMemcpyDeviceToDevice, c->stream));
    if (with_v) SBX_HIP(hipMemcpyAsync(dst.v[k], src.v[k], b, hipMemcpyDeviceToDevice, c->stream));
  }
  if (with_lost) SBX_HIP(hipMemcpyAsync(dst.lost, src.lost, c->n, hipMemcpyDeviceToDevice, c->stream));
  return SBX_OK;
}

// Forward nsteps without sorting, checkpoints of (x, v, lost) every
// ckpt_every steps, then the reverse cycles interval by interval.  The
// positions, lost flags and fields of an interval's cycles are recomputed
// from its checkpoint (the last interval keeps them from the forward pass):
// each cycle's solve runs from the particles that take part in it (live
// after its start-of-step loss test), and its lost flags and fields are kept
// for the reverse cycle, which scatters the adjoint sources, solves them and
// gathers the mass gradient.  A particle lost during the segment thus
// collects dL/dm from the cycles before its loss, and passes its adjoints
// unchanged through the cycles it sat out.  Work arrays live in one device
// buffer of the context, kept between calls.
template <typename T>
sbx_status adjoint_t(sbx_ctx* c, double dt, int nsteps, int ckpt, int sel_comp, int sel_gal,
                     double* loss, double* grad_m, double* grad_x, double* grad_v, bool dev_out) {
  SBX_TRY(ensure_adjoint<T>(c));
  SBX_TRY(set_dt(c, dt));
  const int64_t n = c->n;
  const int nck = (nsteps + ckpt - 1) / ckpt;
  // carve the work buffer: checkpoints (x, v, lost), per-cycle (x, lost) and
  // fields of one interval, adjoint state, loss, staging
  size_t need = 0;
  auto take = [&](size_t bytes) { const size_t at = need; need += (bytes + 255) & ~(size_t)255; return at; };
  std::vector<size_t> ck_off(nck + 1), xb_off(ckpt), fb_off(ckpt);
  const size_t set_x = 3 * sizeof(T) * n;
  for (auto& o : ck_off) o = take(2 * set_x + n);
  for (auto& o : xb_off) o = take(set_x + n);
  for (auto& o : fb_off) o = take(sizeof(T) * c->grid_elems);
  const size_t lx_off = take(sizeof(double) * 3 * n), lv_off = take(sizeof(double) * 3 * n);
  const size_t gm_off = take(sizeof(double) * n), dl_off = take(sizeof(double) * 4);
  const size_t st_off = take(sizeof(double) * 3 * n);
  if (c->adj_work_bytes < need) {
    free_ptr(c->adj_work);
    c->adj_work_bytes = 0;
    SBX_TRY(dev_alloc(&c->adj_work, need));
    c->adj_work_bytes = need;
  }
  char* base = (char*)c->adj_work;
  auto set_at = [&](size_t off, bool with_v, PSet& s) {
    char* q = base + off;
    for (int k = 0; k < 3; ++k) s.x[k] = q + sizeof(T) * n * k;
    q += set_x;
    if (with_v) {
      for (int k = 0; k < 3; ++k) s.v[k] = q + sizeof(T) * n * k;
      q += set_x;
    }
    s.lost = (uint8_t*)q;
  };
  std::vector<PSet> cks(nck + 1), xb(ckpt);
  for (int i = 0; i <= nck; ++i) set_at(ck_off[i], true, cks[i]);
  for (int i = 0; i < ckpt; ++i) set_at(xb_off[i], false, xb[i]);
  double* lx = (double*)(base + lx_off);
  double* lv = (double*)(base + lv_off);
  double* gm = (double*)(base + gm_off);
  double* dloss = (double*)(base + dl_off);
  double* stage = (double*)(base + st_off);
  const size_t gbytes = sizeof(T) * c->grid_elems;
  // reorder by cell once for the segment (locality of the gathers and of
  // the adjoint scatter); nothing is reordered inside the segment
  if (c->sort_every > 0 && !c->bound) SBX_TRY(sort_particles(c));
  PSet& live = c->set[c->cur];
  // one cycle with its record for the reverse: positions before the solve,
  // lost flags after its loss test, fields after the solve
  auto cycle = [&](int slot, bool move) -> sbx_status {
    SBX_TRY(copy_set<T>(c, xb[slot], live, false, false));
    SBX_TRY(field_solve(c));
    SBX_HIP(hipMemcpyAsync(xb[slot].lost, live.lost, n, hipMemcpyDeviceToDevice, c->stream));
    SBX_HIP(hipMemcpyAsync(base + fb_off[slot], c->grid_block, gbytes, hipMemcpyDeviceToDevice, c->stream));
    if (move) SBX_TRY(force(c, 1));
    return SBX_OK;
  };
  // forward with checkpoints; the last interval keeps its records
  const int k0_last = (nck - 1) * ckpt;
  for (int k = 0; k < nsteps; ++k) {
    if (k % ckpt == 0) SBX_TRY(copy_set<T>(c, cks[k / ckpt], live, true, true));
    if (k >= k0_last) {
      SBX_TRY(cycle(k - k0_last, true));
    } else {
      SBX_TRY(field_solve(c));
      SBX_TRY(force(c, 1));
    }
  }
  SBX_TRY(copy_set<T>(c, cks[nck], live, true, true));  // final state
  SBX_TRY(launch_adj_init<T>(dinst<T>(c), c->d_cur, n, sel_comp, sel_gal, lx, lv, gm, c->pre_partial,
                             dloss, c->stream));
  const GridsDev<T> B = adj_grids<T>(c);
  SolvePlan<T>& adj = sizeof(T) == 8 ? (SolvePlan<T>&)c->adj64 : (SolvePlan<T>&)c->adj32;
  for (int seg = nck - 1; seg >= 0; --seg) {
    const int k0 = seg * ckpt, k1 = std::min(k0 + ckpt, nsteps);
    if (seg < nck - 1) {
      SBX_TRY(copy_set<T>(c, live, cks[seg], true, true));
      c->com_fresh = false;  // the first solve runs the start-of-step loss test
      for (int k = k0; k < k1; ++k) SBX_TRY(cycle(k - k0, k + 1 < k1));
    }
    for (int k = k1 - 1; k >= k0; --k) {
      // positions, sat-out flags and forward fields of cycle k
      SBX_TRY(copy_set<T>(c, live, xb[k - k0], false, true));
      SBX_HIP(hipMemcpyAsync(c->grid_block, base + fb_off[k - k0], gbytes, hipMemcpyDeviceToDevice,
                             c->stream));
      SBX_TRY(launch_zero<T>((T*)c->adj_block, c->grid_elems, c->stream));
      SBX_TRY(launch_adj_step<T>(dinst<T>(c), c->d_cur, n, B, live.lost, lx, lv, c->stream));
      SBX_TRY(plan_run<T>(adj, c->stream));
      SBX_TRY(launch_adj_gather<T>(dinst<T>(c), c->d_cur, n, B, live.lost, gm, c->stream));
    }
  }
  SBX_TRY(copy_set<T>(c, live, cks[nck], true, true));  // back to the final state
  c->com_fresh = false;
  c->grids_fields = false;
  c->step_count += nsteps;
  // outputs in the caller's order
  const int32_t* id = live.id;
  if (loss) SBX_HIP(hipMemcpyAsync(loss, dloss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  struct Out { double* host; double* dev; int w; } outs[3] = {{grad_m, gm, 1}, {grad_x, lx, 3}, {grad_v, lv, 3}};
  for (auto& o : outs) {
    if (!o.host) continue;
    SBX_TRY(launch_unpermute<double>(o.dev, id, dev_out ? o.host : stage, n, o.w, c->stream));
    if (!dev_out)
      SBX_HIP(hipMemcpyAsync(o.host, stage, sizeof(double) * o.w * n, hipMemcpyDeviceToHost, c->stream));
    SBX_HIP(hipStreamSynchronize(c->stream));
  }
  SBX_HIP(hipStreamSynchronize(c->stream));
  return SBX_OK;
}

}  // namespace

// ============================================================== the ABI ====
extern "C" {

const char* sbx_last_error(void) { return g_err.c_str(); }

double sbx_q_crit(int32_t n, double R_core, double R_out, double R_sys) {
  return q_crit_of(n, R_core, R_out, R_sys);
}

sbx_status sbx_validate_hierarchies(int32_t n_galaxies, const sbx_hierarchy* h) {
  return validate(n_galaxies, h);
}

sbx_status sbx_create(const sbx_config* cfg, sbx_ctx** out) {
  if (!cfg || !out) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  *out = nullptr;
  if (cfg->prec != SBX_FP32 && cfg->prec != SBX_FP64) {
    set_error("prec must be SBX_FP32 or SBX_FP64");
    return SBX_EINVAL;
  }
  if (cfg->h0_mode < 0 || cfg->h0_mode > 2) {
    set_error("h0_mode must be 0, 1 or 2");
    return SBX_EINVAL;
  }
  if (!std::isfinite(cfg->G) || !(cfg->G > 0.0)) {
    set_error("G must be positive");
    return SBX_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    set_error("no HIP device available");
    return SBX_EDEVICE;
  }
  if (cfg->device < 0 || cfg->device >= ndev) {
    set_error("device ordinal out of range");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(cfg->device));
  sbx_ctx* c = new (std::nothrow) sbx_ctx();
  if (!c) {
    set_error("out of host memory");
    return SBX_ENOMEM;
  }
  c->cfg = *cfg;
  c->esz = cfg->prec == SBX_FP64 ? 8 : 4;
  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      set_error("hipStreamCreate failed");
      return SBX_EDEVICE;
    }
    c->own_stream = true;
  }
  const size_t inst_bytes = cfg->prec == SBX_FP64 ? sizeof(InstDev<double>) : sizeof(InstDev<float>);
  sbx_status rc = SBX_OK;
  if ((rc = dev_alloc((void**)&c->centres, sizeof(double) * 3 * kMaxGal)) != SBX_OK ||
      (rc = dev_alloc((void**)&c->pre_partial, sizeof(double) * ((size_t)kRedBlocks + 1) * kPreVals)) != SBX_OK ||
      (rc = dev_alloc((void**)&c->com_partial, sizeof(double) * (size_t)kForceBlocksMax * kPreVals)) != SBX_OK ||
      (rc = dev_alloc((void**)&c->diag_partial, sizeof(double) * (size_t)kForceBlocksMax * kNDiag)) != SBX_OK ||
      (rc = dev_alloc((void**)&c->diag_one, sizeof(double) * kNDiag)) != SBX_OK ||
      (rc = dev_alloc((void**)&c->diag_log, sizeof(double) * kNDiag * kDiagCap)) != SBX_OK ||
      (rc = dev_alloc(&c->d_inst, inst_bytes)) != SBX_OK ||
      (rc = dev_alloc((void**)&c->d_cur, sizeof(int))) != SBX_OK ||
      (rc = dev_alloc((void**)&c->dm_mmax, sizeof(unsigned long long))) != SBX_OK) {
    sbx_destroy(c);
    return rc;
  }
  *out = c;
  return SBX_OK;
}

void sbx_destroy(sbx_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->cfg.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_particles(c);
  free_grids(c);
  free_typed(c->centres);
  free_typed(c->pre_partial);
  free_typed(c->com_partial);
  free_typed(c->diag_partial);
  free_typed(c->diag_one);
  free_typed(c->diag_log);
  free_typed(c->dm_mmax);
  free_ptr(c->d_inst);
  free_typed(c->d_cur);
  free_recorder(c->rec);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

sbx_status sbx_profile_begin(sbx_ctx* c, int32_t max_marks) {
  if (!c || max_marks <= 0 || max_marks > (1 << 20)) {
    set_error("bad profile arguments");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(c->cfg.device));
  SBX_HIP(hipStreamSynchronize(c->stream));
  if (c->rec.cap < max_marks) {
    free_recorder(c->rec);
    c->rec.ev = new hipEvent_t[max_marks];
    c->rec.tag = new int[max_marks];
    for (int i = 0; i < max_marks; ++i) {
      if (hipEventCreate(&c->rec.ev[i]) != hipSuccess) {
        c->rec.cap = i;
        free_recorder(c->rec);
        set_error("hipEventCreate failed");
        return SBX_EDEVICE;
      }
      c->rec.cap = i + 1;
    }
  }
  c->rec.used = 0;
  c->rec.on = true;
  return SBX_OK;
}

sbx_status sbx_profile_end(sbx_ctx* c, int32_t n_phases, double* out_ms, int64_t* out_count) {
  if (!c || !out_ms || !out_count || n_phases < PH_COUNT) {
    set_error("bad profile arguments");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(c->cfg.device));
  SBX_HIP(hipStreamSynchronize(c->stream));
  for (int i = 0; i < n_phases; ++i) {
    out_ms[i] = 0.0;
    out_count[i] = 0;
  }
  for (int i = 1; i < c->rec.used; ++i) {
    if (c->rec.tag[i] == PH_START) continue;
    float ms = 0.f;
    SBX_HIP(hipEventElapsedTime(&ms, c->rec.ev[i - 1], c->rec.ev[i]));
    out_ms[c->rec.tag[i]] += ms;
    out_count[c->rec.tag[i]] += 1;
  }
  c->rec.on = false;
  c->rec.used = 0;
  return SBX_OK;
}

}  // extern "C"

namespace sbx {

// Whether p is device memory of the given device (device or managed).
bool on_device(const void* p, int device) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged) && at.device == device;
}

sbx_status load_impl(sbx_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                     const int8_t* comp, const int8_t* gal, bool dev) {
  if (!c || n <= 0 || !x || !v || !m || !comp || !gal) {
    set_error("null argument or n <= 0");
    return SBX_EINVAL;
  }
  if (n >= ((int64_t)1 << 31)) {
    set_error("at most 2^31 - 1 particles per context");
    return SBX_EINVAL;
  }
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  SBX_TRY(set_device(c->cfg.device));
  const int ngal_limit = c->built ? c->ngal : kMaxGal;
  if (dev) {
    for (const void* p : {(const void*)x, (const void*)v, (const void*)m, (const void*)comp, (const void*)gal})
      if (!on_device(p, c->cfg.device)) {
        set_error("inputs must be device memory of the context's device");
        return SBX_EINVAL;
      }
    unsigned long long* bad = nullptr;
    SBX_TRY(dev_alloc((void**)&bad, sizeof(unsigned long long)));
    unsigned long long first = ~0ull;
    sbx_status rc = SBX_OK;
    if (hipMemcpyAsync(bad, &first, sizeof(first), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        launch_validate_particles(x, v, m, comp, gal, n, ngal_limit, bad, c->stream) != SBX_OK ||
        hipMemcpyAsync(&first, bad, sizeof(first), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      set_error(std::string("particle validation: ") + hipGetErrorString(hipGetLastError()));
      rc = SBX_EDEVICE;
    }
    (void)hipFree(bad);
    SBX_TRY(rc);
    if (first != ~0ull) {
      set_error("particle " + std::to_string(first) +
                ": masses must be finite and >= 0, positions and velocities finite, component id "
                "in 0..7 and galaxy id within the hierarchies");
      return SBX_EINVAL;
    }
  } else {
    for (int64_t i = 0; i < n; ++i) {
      if (!std::isfinite(m[i]) || m[i] < 0.0) {
        set_error("masses must be finite and >= 0 (particle " + std::to_string(i) + ")");
        return SBX_EINVAL;
      }
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(x[3 * i + k]) || !std::isfinite(v[3 * i + k])) {
          set_error("positions and velocities must be finite (particle " + std::to_string(i) + ")");
          return SBX_EINVAL;
        }
      if (comp[i] < 0 || comp[i] >= kNComp || gal[i] < 0 || gal[i] >= kMaxGal) {
        set_error("component id in 0..7 and galaxy id in 0..7 required");
        return SBX_EINVAL;
      }
      if (c->built && gal[i] >= c->ngal) {
        set_error("galaxy id beyond the built hierarchies");
        return SBX_EINVAL;
      }
    }
  }
  SBX_HIP(hipStreamSynchronize(c->stream));
  free_particles(c);
  const size_t es = c->esz;
  for (int s = 0; s < 2; ++s) {
    PSet& q = c->set[s];
    for (int k = 0; k < 3; ++k) {
      SBX_TRY(dev_alloc(&q.x[k], es * n));
      SBX_TRY(dev_alloc(&q.v[k], es * n));
    }
    SBX_TRY(dev_alloc(&q.m, es * n));
    SBX_TRY(dev_alloc((void**)&q.comp, n));
    SBX_TRY(dev_alloc((void**)&q.gal, n));
    SBX_TRY(dev_alloc((void**)&q.lost, n));
    SBX_TRY(dev_alloc((void**)&q.id, sizeof(int32_t) * n));
  }
  SBX_TRY(dev_alloc((void**)&c->key, sizeof(uint32_t) * n));
  SBX_TRY(dev_alloc((void**)&c->rank, sizeof(uint32_t) * n));
  c->n = n;
  c->cur = 0;
  double* stage = nullptr;
  if (!dev) SBX_TRY(dev_alloc((void**)&stage, sizeof(double) * 3 * n));
  PSet& q = c->set[0];
  // device inputs are read in place; host inputs go through one staging array
  auto in = [&](const double* src, size_t count) -> const double* {
    if (dev) return src;
    if (hipMemcpy(stage, src, sizeof(double) * count, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return stage;
  };
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  auto run = [&]() -> sbx_status {
    for (int which = 0; which < 2; ++which) {
      const double* src = in(which == 0 ? x : v, 3 * (size_t)n);
      if (!src) {
        set_error(std::string("particle upload: ") + hipGetErrorString(hipGetLastError()));
        return SBX_EDEVICE;
      }
      void* const* d = which == 0 ? q.x : q.v;
      if (c->cfg.prec == SBX_FP64)
        SBX_TRY(launch_split3<double>(src, (double*)d[0], (double*)d[1], (double*)d[2], n, c->stream));
      else
        SBX_TRY(launch_split3<float>(src, (float*)d[0], (float*)d[1], (float*)d[2], n, c->stream));
      SBX_HIP(hipStreamSynchronize(c->stream));
    }
    const double* ms = in(m, n);
    if (!ms) {
      set_error(std::string("particle upload: ") + hipGetErrorString(hipGetLastError()));
      return SBX_EDEVICE;
    }
    if (c->cfg.prec == SBX_FP64) {
      SBX_TRY(launch_convert_in<double>(ms, (double*)q.m, n, c->stream));
      SBX_TRY(launch_mass_max<double>((const double*)q.m, n, c->dm_mmax, c->stream));
    } else {
      SBX_TRY(launch_convert_in<float>(ms, (float*)q.m, n, c->stream));
      SBX_TRY(launch_mass_max<float>((const float*)q.m, n, c->dm_mmax, c->stream));
    }
    SBX_HIP(hipMemcpyAsync(q.comp, comp, n, kind, c->stream));
    SBX_HIP(hipMemcpyAsync(q.gal, gal, n, kind, c->stream));
    SBX_TRY(launch_zero<uint8_t>(q.lost, n, c->stream));
    SBX_TRY(launch_iota(q.id, n, c->stream));
    SBX_HIP(hipStreamSynchronize(c->stream));
    return SBX_OK;
  };
  sbx_status rc = run();
  if (stage) (void)hipFree(stage);
  c->solved = false;
  c->grids_fields = false;
  c->com_fresh = false;
  c->step_count = 0;
  if (rc == SBX_OK) rc = upload_inst(c);
  return rc;
}

sbx_status get_impl(sbx_ctx* c, double* x, double* v, uint8_t* lost, bool dev) {
  if (!c || c->n == 0) {
    set_error("no particles loaded");
    return c ? SBX_ESTATE : SBX_EINVAL;
  }
  if (c->batch && c->batch->pending) {
    set_error("the context's batch has queued work: call sbx_batch_sync first");
    return SBX_ESTATE;
  }
  SBX_TRY(set_device(c->cfg.device));
  if (dev)
    for (const void* p : {(const void*)x, (const void*)v, (const void*)lost})
      if (p && !on_device(p, c->cfg.device)) {
        set_error("outputs must be device memory of the context's device");
        return SBX_EINVAL;
      }
  const PSet& q = c->set[c->cur];
  double* stage = nullptr;
  SBX_TRY(dev_alloc((void**)&stage, sizeof(double) * 6 * c->n));
  double* stage2 = stage + 3 * c->n;
  auto run = [&]() -> sbx_status {
    for (int which = 0; which < 2; ++which) {
      double* out = which == 0 ? x : v;
      void* const* src = which == 0 ? q.x : q.v;
      if (!out) continue;
      if (c->cfg.prec == SBX_FP64)
        SBX_TRY(launch_join3<double>((double*)src[0], (double*)src[1], (double*)src[2], stage, c->n, c->stream));
      else
        SBX_TRY(launch_join3<float>((float*)src[0], (float*)src[1], (float*)src[2], stage, c->n, c->stream));
      SBX_TRY(launch_unpermute<double>(stage, q.id, dev ? out : stage2, c->n, 3, c->stream));
      if (!dev) SBX_HIP(hipMemcpyAsync(out, stage2, sizeof(double) * 3 * c->n, hipMemcpyDeviceToHost, c->stream));
      SBX_HIP(hipStreamSynchronize(c->stream));
    }
    if (lost) {
      SBX_TRY(launch_unpermute<uint8_t>(q.lost, q.id, dev ? lost : (uint8_t*)stage, c->n, 1, c->stream));
      if (!dev) SBX_HIP(hipMemcpyAsync(lost, stage, c->n, hipMemcpyDeviceToHost, c->stream));
    }
    SBX_HIP(hipStreamSynchronize(c->stream));
    return SBX_OK;
  };
  const sbx_status rc = run();
  (void)hipFree(stage);
  return rc;
}

// Borrowed particle storage: the caller's structure-of-arrays in the context
// precision becomes the live particle set (never reordered).
template <typename T>
sbx_status bind_t(sbx_ctx* c, int64_t n, void* x, void* v, void* m, int8_t* comp, int8_t* gal,
                  uint8_t* lost) {
  const int ngal_limit = c->built ? c->ngal : kMaxGal;
  unsigned long long* bad = nullptr;
  SBX_TRY(dev_alloc((void**)&bad, sizeof(unsigned long long)));
  unsigned long long first = ~0ull;
  sbx_status rc = SBX_OK;
  if (hipMemcpyAsync(bad, &first, sizeof(first), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      launch_validate_soa<T>((const T*)x, (const T*)v, (const T*)m, comp, gal, n, ngal_limit, bad,
                             c->stream) != SBX_OK ||
      hipMemcpyAsync(&first, bad, sizeof(first), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    set_error(std::string("particle validation: ") + hipGetErrorString(hipGetLastError()));
    rc = SBX_EDEVICE;
  }
  (void)hipFree(bad);
  SBX_TRY(rc);
  if (first != ~0ull) {
    set_error("particle " + std::to_string(first) +
              ": masses must be finite and >= 0, positions and velocities finite, component id "
              "in 0..7 and galaxy id within the hierarchies");
    return SBX_EINVAL;
  }
  free_particles(c);
  PSet& q = c->set[0];
  for (int k = 0; k < 3; ++k) {
    q.x[k] = (T*)x + (size_t)k * n;
    q.v[k] = (T*)v + (size_t)k * n;
  }
  q.m = m;
  q.comp = comp;
  q.gal = gal;
  q.lost = lost;
  c->bound = true;
  c->n = n;
  c->cur = 0;
  if (dev_alloc((void**)&q.id, sizeof(int32_t) * n) != SBX_OK) {
    const std::string msg = sbx_last_error();
    free_particles(c);
    set_error(msg);
    return SBX_ENOMEM;
  }
  SBX_TRY(launch_iota(q.id, n, c->stream));
  SBX_TRY(launch_mass_max<T>((const T*)m, n, c->dm_mmax, c->stream));
  SBX_HIP(hipStreamSynchronize(c->stream));
  c->solved = false;
  c->grids_fields = false;
  c->com_fresh = false;
  c->step_count = 0;
  return upload_inst(c);
}

sbx_status bind_impl(sbx_ctx* c, int64_t n, void* x, void* v, void* m, int8_t* comp, int8_t* gal,
                     uint8_t* lost) {
  if (!c || n <= 0 || !x || !v || !m || !comp || !gal || !lost) {
    set_error("null argument or n <= 0");
    return SBX_EINVAL;
  }
  if (n >= ((int64_t)1 << 31)) {
    set_error("at most 2^31 - 1 particles per context");
    return SBX_EINVAL;
  }
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  SBX_TRY(set_device(c->cfg.device));
  for (const void* p : {(const void*)x, (const void*)v, (const void*)m, (const void*)comp,
                        (const void*)gal, (const void*)lost})
    if (!on_device(p, c->cfg.device)) {
      set_error("bound arrays must be device memory of the context's device");
      return SBX_EINVAL;
    }
  // the moving arrays must not overlap each other or the read-only ones
  const size_t es = c->esz;
  struct Range { uintptr_t a, b; } r[6] = {
      {(uintptr_t)x, (uintptr_t)x + 3 * es * n}, {(uintptr_t)v, (uintptr_t)v + 3 * es * n},
      {(uintptr_t)m, (uintptr_t)m + es * n},     {(uintptr_t)comp, (uintptr_t)comp + n},
      {(uintptr_t)gal, (uintptr_t)gal + n},      {(uintptr_t)lost, (uintptr_t)lost + n}};
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j)
      if ((i < 2 || i == 5 || j < 2 || j == 5) && r[i].a < r[j].b && r[j].a < r[i].b) {
        set_error("the bound positions, velocities and lost flags must not overlap other arrays");
        return SBX_EINVAL;
      }
  SBX_HIP(hipStreamSynchronize(c->stream));
  return c->cfg.prec == SBX_FP64 ? bind_t<double>(c, n, x, v, m, comp, gal, lost)
                                 : bind_t<float>(c, n, x, v, m, comp, gal, lost);
}

}  // namespace sbx

extern "C" {

sbx_status sbx_load_particles(sbx_ctx* c, int64_t n, const double* x, const double* v,
                              const double* m, const int8_t* comp, const int8_t* gal) {
  return load_impl(c, n, x, v, m, comp, gal, false);
}

sbx_status sbx_load_particles_device(sbx_ctx* c, int64_t n, const double* x, const double* v,
                                     const double* m, const int8_t* comp, const int8_t* gal) {
  return load_impl(c, n, x, v, m, comp, gal, true);
}

sbx_status sbx_bind_device_particles(sbx_ctx* c, int64_t n, void* x, void* v, void* m, int8_t* comp,
                                     int8_t* gal, uint8_t* lost) {
  return bind_impl(c, n, x, v, m, comp, gal, lost);
}

sbx_status sbx_build_grids(sbx_ctx* c, int32_t n_galaxies, const sbx_hierarchy* h) {
  if (!c) {
    set_error("null context");
    return SBX_EINVAL;
  }
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  SBX_TRY(validate(n_galaxies, h));
  SBX_TRY(set_device(c->cfg.device));
  SBX_HIP(hipStreamSynchronize(c->stream));
  free_grids(c);
  c->ngal = n_galaxies;
  c->N = h[0].lv[0].n;
  std::memset(&c->sys, 0, sizeof(c->sys));
  c->sys.ngal = n_galaxies;
  c->sys.taylor = c->cfg.taylor ? 1 : 0;
  if (c->merge5) {
    bool ok = n_galaxies >= 2;
    for (int g = 0; g < n_galaxies; ++g) ok = ok && h[g].n_levels == 3;
    if (!ok) {
      set_error("merging the outer grids needs at least two galaxies with three levels");
      return SBX_EINVAL;
    }
    c->sys.merge5 = 1;
  }
  for (int g = 0; g < n_galaxies; ++g) {
    c->hh[g] = h[g];
    HierDev& d = c->sys.h[g];
    d.n_levels = h[g].n_levels;
    d.centring = h[g].centring;
    for (int k = 0; k < h[g].n_levels; ++k) d.lv[k] = make_level(h[g].lv[k]);
    for (int k = 0; k < 3; ++k) {
      d.centre[k] = h[g].centre[k];
      d.outer_c[k] = h[g].outer_centre[k];
    }
    c->nslots[g] = slot_count(h[g]);
    for (int s = 0; s < c->nslots[g]; ++s) c->slot_level[g][s] = slot_level_of(h[g], s);
  }
  sbx_status rc = c->cfg.prec == SBX_FP64 ? build_grids_t<double>(c) : build_grids_t<float>(c);
  if (rc != SBX_OK) {
    free_grids(c);
    return rc;
  }
  c->built = true;
  return upload_inst(c);
}

sbx_status sbx_compute_forces(sbx_ctx* c, double* acc, double* pot) {
  SBX_TRY(check_ready(c));
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  SBX_TRY(ensure_acc(c));
  SBX_TRY(field_solve(c));
  SBX_TRY(force(c, 2));
  const int32_t* id = c->set[c->cur].id;
  double* stage = nullptr;
  SBX_TRY(dev_alloc((void**)&stage, sizeof(double) * 3 * c->n));
  auto run = [&]() -> sbx_status {
    if (acc) {
      SBX_TRY(launch_unpermute<double>(c->acc, id, stage, c->n, 3, c->stream));
      SBX_HIP(hipMemcpyAsync(acc, stage, sizeof(double) * 3 * c->n, hipMemcpyDeviceToHost, c->stream));
      SBX_HIP(hipStreamSynchronize(c->stream));
    }
    if (pot) {
      SBX_TRY(launch_unpermute<double>(c->pot, id, stage, c->n, 1, c->stream));
      SBX_HIP(hipMemcpyAsync(pot, stage, sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
    }
    SBX_HIP(hipStreamSynchronize(c->stream));
    return SBX_OK;
  };
  const sbx_status rc = run();
  (void)hipFree(stage);
  return rc;
}

sbx_status sbx_step(sbx_ctx* c, double dt, int32_t nsteps, int32_t diag_every) {
  SBX_TRY(check_ready(c));
  if (!std::isfinite(dt) || nsteps < 0) {
    set_error("dt must be finite and nsteps >= 0");
    return SBX_EINVAL;
  }
  if (c->batch) {
    set_error("the context belongs to a batch: step it with sbx_batch_step");
    return SBX_ESTATE;
  }
  SBX_TRY(set_dt(c, dt));
  for (int s = 0; s < nsteps; ++s) {
    if (c->sort_every > 0 && !c->bound && (c->step_count % c->sort_every) == 0)
      SBX_TRY(sort_particles(c));
    SBX_TRY(field_solve(c));
    const bool diag = diag_every > 0 && (c->step_count % diag_every) == 0;
    if (diag && c->diag_count < kDiagCap) {
      SBX_TRY(force(c, 1 | 4));
      SBX_HIP(hipMemcpyAsync(c->diag_log + (size_t)kNDiag * c->diag_count, c->diag_one,
                             sizeof(double) * kNDiag, hipMemcpyDeviceToDevice, c->stream));
      ++c->diag_count;
    } else {
      SBX_TRY(force(c, 1));
    }
    ++c->step_count;
  }
  return SBX_OK;
}

sbx_status sbx_get_particles(sbx_ctx* c, double* x, double* v, uint8_t* lost) {
  return get_impl(c, x, v, lost, false);
}

sbx_status sbx_get_particles_device(sbx_ctx* c, double* x, double* v, uint8_t* lost) {
  return get_impl(c, x, v, lost, true);
}

sbx_status sbx_get_centres(sbx_ctx* c, double* centres) {
  SBX_TRY(check_ready(c));
  if (!centres) {
    set_error("null output");
    return SBX_EINVAL;
  }
  if (!c->solved) {
    for (int g = 0; g < c->ngal; ++g)
      for (int k = 0; k < 3; ++k) centres[3 * g + k] = c->hh[g].centre[k];
    return SBX_OK;
  }
  SBX_HIP(hipMemcpyAsync(centres, c->centres, sizeof(double) * 3 * c->ngal, hipMemcpyDeviceToHost,
                         c->stream));
  SBX_HIP(hipStreamSynchronize(c->stream));
  return SBX_OK;
}

sbx_status sbx_get_indices(sbx_ctx* c, int32_t galaxy, int32_t level, int32_t* idx, int8_t* cls) {
  SBX_TRY(check_ready(c));
  if (galaxy < 0 || galaxy >= c->ngal || level < 0 || level >= c->hh[galaxy].n_levels) {
    set_error("galaxy or level out of range");
    return SBX_EINVAL;
  }
  if (!c->solved) {
    // fixed centres until the first solve has computed them
    double hc[3 * kMaxGal];
    for (int g = 0; g < c->ngal; ++g)
      for (int k = 0; k < 3; ++k) hc[3 * g + k] = c->hh[g].centre[k];
    SBX_HIP(hipStreamSynchronize(c->stream));
    SBX_HIP(hipMemcpy(c->centres, hc, sizeof(double) * 3 * c->ngal, hipMemcpyHostToDevice));
  }
  const int32_t* id = c->set[c->cur].id;
  int32_t* di = nullptr;
  int8_t* dc = nullptr;
  SBX_TRY(dev_alloc((void**)&di, sizeof(int32_t) * 6 * c->n));
  if (dev_alloc((void**)&dc, 2 * c->n) != SBX_OK) {
    (void)hipFree(di);
    return SBX_ENOMEM;
  }
  int32_t* di2 = di + 3 * c->n;
  int8_t* dc2 = dc + c->n;
  auto run = [&]() -> sbx_status {
    if (c->cfg.prec == SBX_FP64)
      SBX_TRY(launch_indices<double>(dinst<double>(c), c->d_cur, c->n, galaxy, level, di, dc, c->stream));
    else
      SBX_TRY(launch_indices<float>(dinst<float>(c), c->d_cur, c->n, galaxy, level, di, dc, c->stream));
    SBX_TRY(launch_unpermute<int32_t>(di, id, di2, c->n, 3, c->stream));
    SBX_TRY(launch_unpermute<int8_t>(dc, id, dc2, c->n, 1, c->stream));
    if (idx) SBX_HIP(hipMemcpyAsync(idx, di2, sizeof(int32_t) * 3 * c->n, hipMemcpyDeviceToHost, c->stream));
    if (cls) SBX_HIP(hipMemcpyAsync(cls, dc2, c->n, hipMemcpyDeviceToHost, c->stream));
    SBX_HIP(hipStreamSynchronize(c->stream));
    return SBX_OK;
  };
  const sbx_status rc = run();
  (void)hipFree(di);
  (void)hipFree(dc);
  return rc;
}

sbx_status sbx_get_grid(sbx_ctx* c, int32_t galaxy, int32_t which, int32_t kind, double* out) {
  SBX_TRY(check_ready(c));
  if (galaxy < 0 || galaxy >= c->ngal || which < 0 || which >= field_slot_count(c->hh[galaxy]) || !out ||
      (kind != 0 && kind != 1)) {
    set_error("galaxy, grid or kind out of range");
    return SBX_EINVAL;
  }
  if (!c->solved || (kind == 1 && !c->grids_fields)) {
    set_error("no solve has run since the last change of the grids");
    return SBX_ESTATE;
  }
  const size_t cells = (size_t)c->N * c->N * c->N;
  const std::vector<InstInfo> info{info_of(c)};
  if (kind == 0) {
    // cell masses: re-run the assignment only (the solve overwrote them)
    if (c->cfg.prec == SBX_FP64) {
      SBX_TRY(launch_zero_grids<double>(dinst<double>(c), info, c->stream));
      SBX_TRY(launch_deposit<double>(dinst<double>(c), c->d_cur, info, c->stream));
    } else {
      SBX_TRY(launch_zero_grids<float>(dinst<float>(c), info, c->stream));
      SBX_TRY(launch_deposit<float>(dinst<float>(c), c->d_cur, info, c->stream));
    }
    c->grids_fields = false;
  }
  // masses of the summed grids: their two sources, added here
  const bool sum2 = kind == 0 && c->hh[galaxy].n_levels == 3 && (which == 2 || which == 4);
  const void* src = c->grid[galaxy][which];
  const void* src2 = nullptr;
  if (sum2) {
    src = c->grid[galaxy][which == 2 ? kSlotG2 : kSlotG4];
    if (which == 2 || !c->sys.merge5) src2 = c->grid[galaxy][which == 2 ? 1 : 3];
  }
  double* stage = nullptr;
  SBX_TRY(dev_alloc((void**)&stage, sizeof(double) * cells));
  std::vector<double> add;
  auto fetch = [&](const void* g, double* host) -> sbx_status {
    if (c->cfg.prec == SBX_FP64)
      SBX_TRY(launch_convert_out<double>((const double*)g, stage, cells, c->stream));
    else
      SBX_TRY(launch_convert_out<float>((const float*)g, stage, cells, c->stream));
    SBX_HIP(hipMemcpyAsync(host, stage, sizeof(double) * cells, hipMemcpyDeviceToHost, c->stream));
    SBX_HIP(hipStreamSynchronize(c->stream));
    return SBX_OK;
  };
  auto run = [&]() -> sbx_status {
    SBX_TRY(fetch(src, out));
    if (src2) {
      add.resize(cells);
      SBX_TRY(fetch(src2, add.data()));
      for (size_t i = 0; i < cells; ++i) out[i] += add[i];
    }
    return SBX_OK;
  };
  const sbx_status rc = run();
  (void)hipFree(stage);
  return rc;
}

sbx_status sbx_diagnostics(sbx_ctx* c, double dt, sbx_diag* out) {
  SBX_TRY(check_ready(c));
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  if (!out || !std::isfinite(dt)) {
    set_error("null output or non-finite dt");
    return SBX_EINVAL;
  }
  SBX_TRY(set_dt(c, dt));
  SBX_TRY(field_solve(c));
  SBX_TRY(force(c, 4));
  double r[kNDiag];
  SBX_HIP(hipMemcpyAsync(r, c->diag_one, sizeof(r), hipMemcpyDeviceToHost, c->stream));
  SBX_HIP(hipStreamSynchronize(c->stream));
  to_diag(r, out);
  return SBX_OK;
}

sbx_status sbx_diag_log(sbx_ctx* c, int32_t max, sbx_diag* out, int32_t* count) {
  if (!c || !count || max < 0 || (max > 0 && !out)) {
    set_error("bad argument");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(c->cfg.device));
  *count = (int32_t)c->diag_count;
  const int64_t k = std::min<int64_t>(max, c->diag_count);
  if (k <= 0) return SBX_OK;
  std::vector<double> r((size_t)k * kNDiag);
  SBX_HIP(hipMemcpyAsync(r.data(), c->diag_log, sizeof(double) * r.size(), hipMemcpyDeviceToHost, c->stream));
  SBX_HIP(hipStreamSynchronize(c->stream));
  for (int64_t i = 0; i < k; ++i) to_diag(r.data() + i * kNDiag, out + i);
  return SBX_OK;
}

}  // extern "C"

namespace {

sbx_status adjoint_impl(sbx_ctx* c, double dt, int32_t nsteps, int32_t ckpt_every, int32_t sel_comp,
                        int32_t sel_gal, double* loss, double* grad_m, double* grad_x,
                        double* grad_v, bool dev_out) {
  SBX_TRY(check_ready(c));
  if (dev_out)
    for (const void* p : {(const void*)grad_m, (const void*)grad_x, (const void*)grad_v})
      if (p && !on_device(p, c->cfg.device)) {
        set_error("gradient outputs must be device memory of the context's device");
        return SBX_EINVAL;
      }
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  if (!std::isfinite(dt) || nsteps < 1 || ckpt_every < 1 || sel_comp < 0 || sel_comp >= kNComp ||
      sel_gal < 0 || sel_gal >= c->ngal) {
    set_error("bad segment arguments");
    return SBX_EINVAL;
  }
  for (int g = 0; g < c->ngal; ++g)
    if (c->hh[g].centring != SBX_CENTRE_FIXED) {
      set_error("the segment adjoint needs fixed centres");
      return SBX_EINVAL;
    }
  if (c->sys.merge5) {
    set_error("the segment adjoint needs separate outer grids (no sbx_set_outer_merge)");
    return SBX_EINVAL;
  }
  return c->cfg.prec == SBX_FP64
             ? adjoint_t<double>(c, dt, nsteps, ckpt_every, sel_comp, sel_gal, loss, grad_m, grad_x,
                                 grad_v, dev_out)
             : adjoint_t<float>(c, dt, nsteps, ckpt_every, sel_comp, sel_gal, loss, grad_m, grad_x,
                                grad_v, dev_out);
}

}  // namespace

extern "C" {

sbx_status sbx_adjoint_segment(sbx_ctx* c, double dt, int32_t nsteps, int32_t ckpt_every,
                               int32_t sel_comp, int32_t sel_gal, double* loss, double* grad_m,
                               double* grad_x, double* grad_v) {
  return adjoint_impl(c, dt, nsteps, ckpt_every, sel_comp, sel_gal, loss, grad_m, grad_x, grad_v, false);
}

sbx_status sbx_adjoint_segment_device(sbx_ctx* c, double dt, int32_t nsteps, int32_t ckpt_every,
                                      int32_t sel_comp, int32_t sel_gal, double* loss,
                                      double* grad_m, double* grad_x, double* grad_v) {
  return adjoint_impl(c, dt, nsteps, ckpt_every, sel_comp, sel_gal, loss, grad_m, grad_x, grad_v, true);
}

sbx_status sbx_set_outer_merge(sbx_ctx* c, int32_t merge) {
  if (!c || (merge != 0 && merge != 1)) {
    set_error("bad argument");
    return SBX_EINVAL;
  }
  c->merge5 = merge;
  return SBX_OK;
}

sbx_status sbx_set_deterministic_deposit(sbx_ctx* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) {
    set_error("bad argument");
    return SBX_EINVAL;
  }
  if (c->batch) {
    set_error("the context belongs to a batch");
    return SBX_ESTATE;
  }
  SBX_TRY(set_device(c->cfg.device));
  c->fix_on = on != 0;
  if (c->fix_on && !c->fix && c->grid_block) {
    SBX_TRY(dev_alloc((void**)&c->fix, sizeof(unsigned long long) * c->mass_elems));
    SBX_HIP(hipMemsetAsync(c->fix, 0, sizeof(unsigned long long) * c->mass_elems, c->stream));
  } else if (!c->fix_on && c->fix) {
    SBX_HIP(hipStreamSynchronize(c->stream));  // no kernel in flight still uses them
    free_typed(c->fix);
  }
  return upload_inst(c);
}

sbx_status sbx_set_sort_interval(sbx_ctx* c, int32_t every) {
  if (!c || every < 0) {
    set_error("bad argument");
    return SBX_EINVAL;
  }
  c->sort_every = every;
  return SBX_OK;
}

sbx_status sbx_sync(sbx_ctx* c) {
  if (!c) {
    set_error("null context");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(c->cfg.device));
  SBX_HIP(hipStreamSynchronize(c->stream));
  return SBX_OK;
}

sbx_status sbx_get_counts(sbx_ctx* c, int64_t* n, int32_t* n_galaxies) {
  if (!c) {
    set_error("null context");
    return SBX_EINVAL;
  }
  if (n) *n = c->n;
  if (n_galaxies) *n_galaxies = c->built ? c->ngal : 0;
  return SBX_OK;
}

sbx_status sbx_count_live(sbx_ctx* c, int64_t* live) {
  if (!c || !live) {
    set_error("null argument");
    return SBX_EINVAL;
  }
  if (c->n == 0) {
    *live = 0;
    return SBX_OK;
  }
  SBX_TRY(set_device(c->cfg.device));
  std::vector<uint8_t> l((size_t)c->n);
  SBX_HIP(hipMemcpyAsync(l.data(), c->set[c->cur].lost, c->n, hipMemcpyDeviceToHost, c->stream));
  SBX_HIP(hipStreamSynchronize(c->stream));
  int64_t k = 0;
  for (uint8_t b : l) k += b ? 0 : 1;
  *live = k;
  return SBX_OK;
}

}  // extern "C"
