// C ABI of batches: several independent contexts (instances) stepped
// together.  Every phase of a step is one launch over all instances (the
// FFT passes: one launch per distinct grid size), and a step is replayed as
// one captured HIP graph.
#include "ctx.h"

using namespace sbx;

namespace {

template <typename T>
SolvePlan<T>& bplan(sbx_batch* b) {
  if constexpr (sizeof(T) == 8) return b->p64;
  else return b->p32;
}

template <typename T>
const SolvePlan<T>& cplan(const sbx_ctx* c) {
  if constexpr (sizeof(T) == 8) return c->plan64;
  else return c->plan32;
}

template <typename T>
sbx_status upload_table(sbx_batch* b) {
  SBX_HIP(hipStreamSynchronize(b->stream));
  std::vector<InstDev<T>> tab(b->ctx.size());
  size_t coff = 0;
  uint32_t pbase = 0;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    sbx_ctx* c = b->ctx[i];
    c->dt_dev = b->dt[i];
    tab[i] = inst_of<T>(c);
    tab[i].count = b->counts + coff;
    tab[i].part_base = pbase;
    coff += c->bins + 1;
    pbase += (uint32_t)c->n;
  }
  SBX_HIP(hipMemcpy(b->d_inst, tab.data(), sizeof(InstDev<T>) * tab.size(), hipMemcpyHostToDevice));
  std::vector<int> cur(b->ctx.size(), b->cur);
  SBX_HIP(hipMemcpy(b->d_cur, cur.data(), sizeof(int) * cur.size(), hipMemcpyHostToDevice));
  return SBX_OK;
}

template <typename T>
sbx_status record_step(sbx_batch* b, bool from_com, bool with_sort) {
  const InstDev<T>* inst = (const InstDev<T>*)b->d_inst;
  if (with_sort)
    SBX_TRY(launch_sort<T>(inst, b->d_cur, b->info, b->counts, b->total_counts, b->scan_tmp, b->stream));
  bool any_dm = false;
  for (const InstInfo& f : b->info) any_dm = any_dm || f.dm_elems > 0;
  if (from_com && !any_dm) {
    SBX_TRY(launch_zero_and_centres<T>(inst, b->info, b->stream));
  } else {
    SBX_TRY(launch_zero_grids<T>(inst, b->info, b->stream));
    SBX_TRY(launch_centres<T>(inst, b->d_cur, b->info, from_com, b->stream));
  }
  SBX_TRY(launch_deposit<T>(inst, b->d_cur, b->info, b->stream));
  SBX_TRY(plan_run<T>(bplan<T>(b), b->stream));
  SBX_TRY(launch_force<T>(inst, b->d_cur, b->info, 1, b->stream));
  return SBX_OK;
}

template <typename T>
sbx_status capture(sbx_batch* b, int which) {
  SBX_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const sbx_status rc = record_step<T>(b, true, which == 1);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != SBX_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
    return SBX_EDEVICE;
  }
  b->graph[which] = g;
  SBX_HIP(hipGraphInstantiate(&b->exec[which], g, nullptr, nullptr, 0));
  return SBX_OK;
}

template <typename T>
sbx_status create_t(sbx_batch* b) {
  b->info.clear();
  b->total_counts = 0;
  std::vector<SolveDesc<T>> descs;
  for (sbx_ctx* c : b->ctx) {
    b->info.push_back(info_of(c));
    b->total_counts += c->bins + 1;
    const SolvePlan<T>& cp = cplan<T>(c);
    descs.insert(descs.end(), cp.host.begin(), cp.host.end());
  }
  if (b->total_counts >= ((size_t)1 << 32)) {
    set_error("too many sort bins in one batch");
    return SBX_EINVAL;
  }
  SBX_TRY(dev_alloc(&b->d_inst, sizeof(InstDev<T>) * b->ctx.size()));
  SBX_TRY(dev_alloc((void**)&b->d_cur, sizeof(int) * b->ctx.size()));
  SBX_TRY(dev_alloc((void**)&b->counts, sizeof(uint32_t) * b->total_counts));
  SBX_TRY(dev_alloc((void**)&b->scan_tmp, sizeof(uint32_t) * scan_tmp_elems(b->total_counts)));
  SBX_TRY(plan_create<T>(bplan<T>(b), descs.data(), (int)descs.size(), b->stream));
  return upload_table<T>(b);
}

template <typename T>
sbx_status step_t(sbx_batch* b, int nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    const bool with_sort = b->sort_every > 0 && (b->step_count % b->sort_every) == 0;
    if (!b->fresh) {
      // first step: loss test and centres from the particles themselves
      SBX_TRY(record_step<T>(b, false, with_sort));
      b->fresh = true;
    } else {
      const int w = with_sort ? 1 : 0;
      if (!b->exec[w]) SBX_TRY(capture<T>(b, w));
      SBX_HIP(hipGraphLaunch(b->exec[w], b->stream));
    }
    if (with_sort) b->cur ^= 1;
    ++b->step_count;
  }
  return SBX_OK;
}

void release(sbx_batch* b) {
  for (int w = 0; w < 2; ++w) {
    if (b->exec[w]) (void)hipGraphExecDestroy(b->exec[w]);
    if (b->graph[w]) (void)hipGraphDestroy(b->graph[w]);
    b->exec[w] = nullptr;
    b->graph[w] = nullptr;
  }
  plan_destroy(b->p32);
  plan_destroy(b->p64);
  free_ptr(b->d_inst);
  if (b->d_cur) (void)hipFree(b->d_cur);
  if (b->counts) (void)hipFree(b->counts);
  if (b->scan_tmp) (void)hipFree(b->scan_tmp);
  b->d_cur = nullptr;
  b->counts = nullptr;
  b->scan_tmp = nullptr;
}

// Hand the batch state back to the member contexts (after a sync).
sbx_status write_back(sbx_batch* b) {
  for (sbx_ctx* c : b->ctx) {
    c->cur = b->cur;
    c->com_fresh = b->fresh;
    c->solved = c->solved || b->step_count > 0;
    c->grids_fields = false;
    c->step_count = b->step_count;
    SBX_HIP(hipMemcpy(c->d_cur, &c->cur, sizeof(int), hipMemcpyHostToDevice));
  }
  return SBX_OK;
}

}  // namespace

extern "C" {

sbx_status sbx_batch_create(sbx_ctx* const* ctxs, int32_t n, void* stream, sbx_batch** out) {
  if (!ctxs || !out || n <= 0 || n > kMaxInst) {
    set_error("1 to 32 contexts per batch");
    return SBX_EINVAL;
  }
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    sbx_ctx* c = ctxs[i];
    if (!c || !c->built || c->n == 0) {
      set_error("every context needs built grids and loaded particles");
      return SBX_ESTATE;
    }
    if (c->batch) {
      set_error("a context already belongs to a batch");
      return SBX_ESTATE;
    }
    if (c->bound) {
      set_error("a context with bound (borrowed) particles cannot join a batch: the batch "
                "reorders particles");
      return SBX_ESTATE;
    }
    if (c->cfg.prec != ctxs[0]->cfg.prec || c->cfg.device != ctxs[0]->cfg.device) {
      set_error("contexts of a batch share device and precision");
      return SBX_EINVAL;
    }
    if ((c->fix != nullptr) != (ctxs[0]->fix != nullptr)) {
      set_error("contexts of a batch share the mass assignment form (fixed-point or not)");
      return SBX_EINVAL;
    }
    if (c->cur != ctxs[0]->cur || c->com_fresh != ctxs[0]->com_fresh) {
      set_error("contexts of a batch must be in the same state (fresh, or all stepped together)");
      return SBX_ESTATE;
    }
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) {
        set_error("a context appears twice");
        return SBX_EINVAL;
      }
  }
  SBX_TRY(set_device(ctxs[0]->cfg.device));
  for (int i = 0; i < n; ++i) SBX_HIP(hipStreamSynchronize(ctxs[i]->stream));
  sbx_batch* b = new (std::nothrow) sbx_batch();
  if (!b) return SBX_ENOMEM;
  b->ctx.assign(ctxs, ctxs + n);
  b->prec = ctxs[0]->cfg.prec;
  b->device = ctxs[0]->cfg.device;
  b->cur = ctxs[0]->cur;
  b->fresh = ctxs[0]->com_fresh;
  b->sort_every = ctxs[0]->sort_every;
  b->step_count = ctxs[0]->step_count;
  for (int i = 0; i < n; ++i) b->dt.push_back(ctxs[i]->dt_dev);
  if (stream) {
    b->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      delete b;
      set_error("hipStreamCreate failed");
      return SBX_EDEVICE;
    }
    b->own_stream = true;
  }
  const sbx_status rc = b->prec == SBX_FP64 ? create_t<double>(b) : create_t<float>(b);
  if (rc != SBX_OK) {
    release(b);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return rc;
  }
  for (sbx_ctx* c : b->ctx) c->batch = b;
  *out = b;
  return SBX_OK;
}

sbx_status sbx_batch_step(sbx_batch* b, const double* dt, int32_t nsteps) {
  if (!b || nsteps < 0) {
    set_error("bad batch step arguments");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(b->device));
  if (dt) {
    bool changed = false;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
      if (!std::isfinite(dt[i])) {
        set_error("dt must be finite");
        return SBX_EINVAL;
      }
      changed = changed || dt[i] != b->dt[i];
    }
    if (changed) {
      b->dt.assign(dt, dt + b->ctx.size());
      SBX_TRY(b->prec == SBX_FP64 ? upload_table<double>(b) : upload_table<float>(b));
    }
  }
  b->pending = true;
  return b->prec == SBX_FP64 ? step_t<double>(b, nsteps) : step_t<float>(b, nsteps);
}

sbx_status sbx_batch_sync(sbx_batch* b) {
  if (!b) {
    set_error("null batch");
    return SBX_EINVAL;
  }
  SBX_TRY(set_device(b->device));
  SBX_HIP(hipStreamSynchronize(b->stream));
  SBX_TRY(write_back(b));
  b->pending = false;
  return SBX_OK;
}

sbx_status sbx_batch_set_sort_interval(sbx_batch* b, int32_t every) {
  if (!b || every < 0) {
    set_error("bad argument");
    return SBX_EINVAL;
  }
  b->sort_every = every;
  return SBX_OK;
}

void sbx_batch_destroy(sbx_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  (void)write_back(b);
  for (sbx_ctx* c : b->ctx) {
    c->batch = nullptr;
    for (size_t i = 0; i < b->ctx.size(); ++i)
      if (b->ctx[i] == c) c->dt_dev = b->dt[i];
    (void)upload_inst(c);
  }
  release(b);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
