// Runtime of the batched form: many independent control problems of uneven
// size advanced together by persistent launches, one gradient iteration
// captured in a HIP graph and replayed, tile shape and residency chosen by
// a timing autotuner.  See include/mrt.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "batch_internal.h"
#include "mrt.h"

namespace {

using mrt::BatchArgs;
using mrt::BatchTile;

int err(int code, const std::string& m) { return mrt::host::set_error(code, m.c_str()); }

#define HIP_OK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return err(MRT_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct mrt_batch {
  int count = 0, dtype = 0, N = 0, K = 0, nseg = 1, mode = 1, device = 0;
  size_t elem = 4, F = 0;
  std::vector<int> L;
  std::vector<size_t> foff;
  std::vector<mrt_problem> probs;
  std::vector<void*> allocs;
  // device data
  char* fields = nullptr;  // 8 fields of F elements: u0 v0 c ut uN vN seed grad
  double* gacc = nullptr;
  void* buf[2] = {nullptr, nullptr};
  void* abuf[2] = {nullptr, nullptr};
  void* ckpt = nullptr;
  void* rec = nullptr;
  void* coef = nullptr;
  int* dL = nullptr;
  size_t* dfoff = nullptr;
  double* dalpha = nullptr;
  BatchTile* tiles = nullptr;
  int* tbeg = nullptr;
  size_t tile_cap = 0;
  int ntiles = 0, tile_w = 64, bpc = 0, max_bpc_f = 0, max_bpc_a = 0, n_cu = 0;
  double* partials = nullptr;
  double* res_cost = nullptr;
  double* res_grad = nullptr;
  double* host = nullptr;  // pinned: 2 * count * kBatchSlots + 1
  mrt::BarrierState* barrier = nullptr;
  unsigned long long timeout = 0, clock_khz = 0;
  // graph
  hipStream_t ps = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_valid = false;
  double graph_zeta = 0.0;
  bool iterated = false;
};

namespace {

char* field_ptr(mrt_batch* b, int which) {
  return b->fields + size_t(which) * b->F * b->elem;
}

template <typename T>
BatchArgs<T> make_args(mrt_batch* b) {
  BatchArgs<T> a{};
  a.tiles = b->tiles;
  a.ntiles = b->ntiles;
  a.tile_w = b->tile_w;
  a.coef = static_cast<const mrt::ModelCoef<T>*>(b->coef);
  a.L = b->dL;
  a.foff = b->dfoff;
  a.alpha = b->dalpha;
  a.N = b->N;
  a.K = b->K;
  a.nseg = b->nseg;
  a.mode = b->mode;
  a.rec_seg = b->nseg - 1;
  a.state_elems = 18 * b->F;
  a.rec_elems = 3 * b->F;
  a.buf[0] = static_cast<T*>(b->buf[0]);
  a.buf[1] = static_cast<T*>(b->buf[1]);
  a.abuf[0] = static_cast<T*>(b->abuf[0]);
  a.abuf[1] = static_cast<T*>(b->abuf[1]);
  a.ckpt = static_cast<T*>(b->ckpt);
  a.rec = static_cast<T*>(b->rec);
  a.u0 = reinterpret_cast<const T*>(field_ptr(b, MRT_FIELD_U0));
  a.v0 = reinterpret_cast<const T*>(field_ptr(b, MRT_FIELD_V0));
  a.ctrl = reinterpret_cast<T*>(field_ptr(b, MRT_FIELD_CONTROL));
  a.ut = reinterpret_cast<const T*>(field_ptr(b, MRT_FIELD_TARGET));
  a.uN = reinterpret_cast<T*>(field_ptr(b, MRT_FIELD_UN));
  a.vN = reinterpret_cast<T*>(field_ptr(b, MRT_FIELD_VN));
  a.grad = reinterpret_cast<T*>(field_ptr(b, MRT_FIELD_GRAD));
  a.seed_u = reinterpret_cast<T*>(field_ptr(b, 7));
  a.gacc = b->gacc;
  a.barrier = b->barrier;
  a.timeout = b->timeout;
  return a;
}

int build_tiles(mrt_batch* b, int tile_w) {
  if (tile_w != 64 && tile_w != 128 && tile_w != 256)
    return err(MRT_EINVAL, "tile_w must be 64, 128 or 256");
  const int tile_h = 256 / tile_w;
  std::vector<BatchTile> t;
  std::vector<int> beg(b->count + 1, 0);
  for (int k = 0; k < b->count; ++k) {
    beg[k] = int(t.size());
    for (int y = 0; y < b->L[k]; y += tile_h)
      for (int x = 0; x < b->L[k]; x += tile_w)
        t.push_back({k, y, x, b->L[k], (unsigned long long)b->foff[k], 0ull});
  }
  beg[b->count] = int(t.size());
  if (t.size() > b->tile_cap) return err(MRT_EINVAL, "tile table overflow");
  HIP_OK(hipMemcpy(b->tiles, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(b->tbeg, beg.data(), beg.size() * sizeof(int), hipMemcpyHostToDevice));
  b->ntiles = int(t.size());
  b->tile_w = tile_w;
  b->graph_valid = false;
  return MRT_OK;
}

int persistent_blocks(const mrt_batch* b, int max_bpc) {
  const int bpc = std::max(1, std::min(b->bpc > 0 ? b->bpc : max_bpc, max_bpc));
  return std::max(1, std::min(b->ntiles, b->n_cu * bpc));
}

int launch_error() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return err(MRT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MRT_OK;
}

// Enqueue one gradient iteration for every instance on stream s.
template <typename T>
int enqueue_iteration(mrt_batch* b, double zeta, hipStream_t s) {
  BatchArgs<T> a = make_args<T>(b);
  const int bf = persistent_blocks(b, b->max_bpc_f);
  const int ba = persistent_blocks(b, b->max_bpc_a);
  const int bs = std::min(b->ntiles, 4096);
  mrt::launch_batch_forward<T>(a, bf, s);
  // the last forward state is buf[(N-1) & 1] (the final step never closes a
  // checkpoint segment)
  mrt::launch_batch_finalize<T>(a, static_cast<const T*>(b->buf[(b->N - 1) & 1]), bs, s);
  mrt::launch_batch_cost<T>(a, 1, b->partials, b->tbeg, b->res_cost, b->count, bs, s);
  mrt::launch_batch_adjoint<T>(a, ba, s);
  mrt::launch_batch_cost<T>(a, 2, b->partials, b->tbeg, b->res_grad, b->count, bs, s);
  mrt::launch_batch_gd<T>(a, zeta, b->res_grad, bs, s);
  return launch_error();
}

int enqueue(mrt_batch* b, double zeta, hipStream_t s) {
  return b->dtype == MRT_F64 ? enqueue_iteration<double>(b, zeta, s)
                             : enqueue_iteration<float>(b, zeta, s);
}

void free_batch(mrt_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->ps) (void)hipStreamDestroy(b->ps);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->host) (void)hipHostFree(b->host);
  delete b;
}

template <typename T>
int upload_coefs(mrt_batch* b) {
  std::vector<mrt::ModelCoef<T>> c(b->count);
  for (int k = 0; k < b->count; ++k) c[k] = mrt::host::model_coef<T>(&b->probs[k]);
  HIP_OK(hipMemcpy(b->coef, c.data(), c.size() * sizeof(c[0]), hipMemcpyHostToDevice));
  return MRT_OK;
}

}  // namespace

extern "C" {

int mrt_batch_create(const mrt_problem* problems, int32_t count,
                     int32_t ckpt_every, size_t mem_budget, mrt_batch** out) {
  if (!out) return err(MRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!problems || count < 1) return err(MRT_EINVAL, "need at least one problem");
  const mrt_grid& g0 = problems[0].grid;
  for (int k = 0; k < count; ++k) {
    const mrt_problem* p = &problems[k];
    int rc = mrt::host::validate(p);
    if (rc) return rc;
    const mrt_grid& g = p->grid;
    if (!g.periodic || g.mask || g.nx != g.ny || g.pitch != g.nx)
      return err(MRT_EINVAL, "batched problems must be periodic, unmasked, square, pitch == nx");
    if (g.dtype != g0.dtype || g.nsteps != g0.nsteps)
      return err(MRT_EINVAL, "batched problems must share dtype and nsteps");
    if (p->source_term > 1)
      return err(MRT_EINVAL, "the batched engine runs the first-order source term only");
    if (p->nspecies == 3)
      return err(MRT_EINVAL, "the batched engine runs two species only");
  }
  mrt_batch* b = new mrt_batch();
  b->count = count;
  b->dtype = g0.dtype;
  b->elem = g0.dtype == MRT_F64 ? 8 : 4;
  b->N = g0.nsteps;
  b->probs.assign(problems, problems + count);
  size_t ntile_max = 0;
  for (int k = 0; k < count; ++k) {
    b->L.push_back(problems[k].grid.nx);
    b->foff.push_back(b->F);
    b->F += size_t(problems[k].grid.nx) * problems[k].grid.nx;
    const size_t Lk = size_t(problems[k].grid.nx);
    size_t most = 0;  // partial tiles make the widest tiles the most numerous on small lattices
    for (size_t w : {64, 128, 256}) most = std::max(most, ((Lk + w - 1) / w) * ((Lk + 256 / w - 1) / (256 / w)));
    ntile_max += most;
  }
  if (ckpt_every < 0) {  // forward solves only: no adjoint buffers, no record
    b->mode = 0;
    b->K = b->N;
    b->nseg = 1;
  } else if (ckpt_every == 0 || ckpt_every >= b->N) {
    b->mode = 1;
    b->K = b->N;
    b->nseg = 1;
  } else {
    b->mode = 2;
    b->K = ckpt_every;
    b->nseg = (b->N + ckpt_every - 1) / ckpt_every;
  }
  const size_t state = 18 * b->F * b->elem;
  const bool adj = b->mode > 0;
  const size_t total = 8 * b->F * b->elem + b->F * 8 + (adj ? 4 : 2) * state +
                       size_t(b->nseg - 1) * state +
                       (adj ? size_t(b->K) * 3 * b->F * b->elem : 0);
  if (mem_budget > 0 && total > mem_budget) {
    delete b;
    return err(MRT_ENOMEM, "batch needs " + std::to_string(total) + " bytes, over the budget");
  }
  auto alloc = [&](size_t bytes, void** p) -> int {
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return err(MRT_ENOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed");
    }
    b->allocs.push_back(*p);
    return MRT_OK;
  };
  int rc = MRT_OK;
  if (hipGetDevice(&b->device) != hipSuccess) rc = err(MRT_EHIP, "no device");
  if (!rc) rc = alloc(8 * b->F * b->elem, (void**)&b->fields);
  if (!rc) rc = alloc(b->F * sizeof(double), (void**)&b->gacc);
  for (int i = 0; i < 2 && !rc; ++i) rc = alloc(state, &b->buf[i]);
  for (int i = 0; i < 2 && !rc && adj; ++i) rc = alloc(state, &b->abuf[i]);
  if (!rc && b->nseg > 1) rc = alloc(size_t(b->nseg - 1) * state, &b->ckpt);
  if (!rc && adj) rc = alloc(size_t(b->K) * 3 * b->F * b->elem, &b->rec);
  if (!rc) rc = alloc(size_t(count) * sizeof(mrt::ModelCoef<double>), &b->coef);
  if (!rc) rc = alloc(count * sizeof(int), (void**)&b->dL);
  if (!rc) rc = alloc(count * sizeof(size_t), (void**)&b->dfoff);
  if (!rc) rc = alloc(count * sizeof(double), (void**)&b->dalpha);
  b->tile_cap = ntile_max;
  if (!rc) rc = alloc(ntile_max * sizeof(BatchTile), (void**)&b->tiles);
  if (!rc) rc = alloc((count + 1) * sizeof(int), (void**)&b->tbeg);
  if (!rc) rc = alloc(ntile_max * mrt::kRedSlots * sizeof(double), (void**)&b->partials);
  if (!rc) rc = alloc(size_t(count) * mrt::kBatchSlots * sizeof(double), (void**)&b->res_cost);
  if (!rc) rc = alloc(size_t(count) * mrt::kBatchSlots * sizeof(double), (void**)&b->res_grad);
  if (!rc) rc = alloc(sizeof(mrt::BarrierState), (void**)&b->barrier);
  if (!rc && hipHostMalloc((void**)&b->host, (2 * size_t(count) * mrt::kBatchSlots + 8) *
                                                 sizeof(double)) != hipSuccess)
    rc = err(MRT_ENOMEM, "hipHostMalloc failed");
  if (rc) {
    free_batch(b);
    return rc;
  }
  std::vector<double> alpha(count);
  for (int k = 0; k < count; ++k) alpha[k] = problems[k].alpha;
  int cu = 0, khz = 0;
  hipError_t e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device);
  if (e == hipSuccess) e = hipMemcpy(b->dL, b->L.data(), count * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->dfoff, b->foff.data(), count * sizeof(size_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->dalpha, alpha.data(), count * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->fields, 0, 8 * b->F * b->elem);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->ps, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    rc = err(MRT_EHIP, std::string("batch set-up: ") + hipGetErrorString(e));
    free_batch(b);
    return rc;
  }
  b->n_cu = cu;
  b->clock_khz = (unsigned long long)std::max(khz, 1);
  b->timeout = b->clock_khz * 2000ull;  // 2 s
  rc = b->dtype == MRT_F64 ? upload_coefs<double>(b) : upload_coefs<float>(b);
  if (!rc) {
    b->max_bpc_f = b->dtype == MRT_F64 ? mrt::batch_max_blocks_per_cu<double>(0)
                                       : mrt::batch_max_blocks_per_cu<float>(0);
    b->max_bpc_a = b->dtype == MRT_F64 ? mrt::batch_max_blocks_per_cu<double>(1)
                                       : mrt::batch_max_blocks_per_cu<float>(1);
    if (b->max_bpc_f < 1 || b->max_bpc_a < 1) rc = err(MRT_EHIP, "occupancy query failed");
  }
  if (!rc) rc = build_tiles(b, 64);
  if (!rc) {
    mrt::launch_barrier_reset(b->barrier, nullptr);
    rc = launch_error();
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = err(MRT_EHIP, "set-up sync failed");
  }
  if (rc) {
    free_batch(b);
    return rc;
  }
  *out = b;
  return MRT_OK;
}

void mrt_batch_destroy(mrt_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_batch(b);
}

int mrt_batch_field(mrt_batch* b, int32_t k, int32_t which, void** ptr) {
  if (!b || !ptr) return err(MRT_EINVAL, "NULL argument");
  if (k < 0 || k >= b->count) return err(MRT_EINVAL, "instance out of range");
  if (which < MRT_FIELD_U0 || which > MRT_FIELD_GRAD) return err(MRT_EINVAL, "unknown field");
  *ptr = field_ptr(b, which) + b->foff[k] * b->elem;
  return MRT_OK;
}

int mrt_batch_copy(mrt_batch* b, int32_t k, int32_t which, int32_t to_batch,
                   void* data, void* stream) {
  void* f = nullptr;
  int rc = mrt_batch_field(b, k, which, &f);
  if (rc) return rc;
  if (!data) return err(MRT_EINVAL, "data is NULL");
  const size_t bytes = size_t(b->L[k]) * b->L[k] * b->elem;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (to_batch)
    HIP_OK(hipMemcpyAsync(f, data, bytes, hipMemcpyDeviceToDevice, s));
  else
    HIP_OK(hipMemcpyAsync(data, f, bytes, hipMemcpyDeviceToDevice, s));
  if (to_batch && which == MRT_FIELD_CONTROL) b->iterated = false;
  return MRT_OK;
}

int mrt_batch_set_tiles(mrt_batch* b, const mrt_batch_tiles* tiles) {
  if (!b || !tiles) return err(MRT_EINVAL, "NULL argument");
  const int maxb = std::min(b->max_bpc_f, b->max_bpc_a);
  if (tiles->blocks_per_cu < 1 || tiles->blocks_per_cu > maxb)
    return err(MRT_EINVAL, "blocks_per_cu outside 1.." + std::to_string(maxb));
  int rc = build_tiles(b, tiles->tile_w);
  if (rc) return rc;
  b->bpc = tiles->blocks_per_cu;
  return MRT_OK;
}

int mrt_batch_get_tiles(mrt_batch* b, mrt_batch_tiles* tiles) {
  if (!b || !tiles) return err(MRT_EINVAL, "NULL argument");
  tiles->tile_w = b->tile_w;
  tiles->blocks_per_cu = b->bpc > 0 ? b->bpc : std::min(b->max_bpc_f, b->max_bpc_a);
  tiles->max_blocks_per_cu = std::min(b->max_bpc_f, b->max_bpc_a);
  tiles->ms_per_step = 0.0;
  return MRT_OK;
}

int mrt_batch_tune(mrt_batch* b, int32_t steps, mrt_batch_tiles* best,
                   void* stream) {
  if (!b || steps < 2) return err(MRT_EINVAL, "need a batch and steps >= 2");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const int maxb = std::min(b->max_bpc_f, b->max_bpc_a);
  double best_ms = 1e300;
  int best_w = 64, best_b = maxb;
  int rc = MRT_OK;
  for (int w : {64, 128, 256}) {
    rc = build_tiles(b, w);
    if (rc) break;
    for (int bpc = 1; bpc <= maxb; bpc *= 2) {
      b->bpc = bpc;
      // one warm-up pass, then the fastest of three timed passes (a single
      // pass of a few milliseconds varies by a few percent, which is the
      // gap between neighbouring shapes)
      double ms_best = 1e300;
      for (int rep = 0; rep < 4 && !rc; ++rep) {
        // forward-only pass of `steps` steps (no record, no checkpoints)
        float ms = 0.f;
        if (b->dtype == MRT_F64) {
          BatchArgs<double> a = make_args<double>(b);
          a.N = steps; a.K = steps; a.nseg = 1; a.mode = 0;
          (void)hipEventRecord(e0, s);
          mrt::launch_batch_forward<double>(a, persistent_blocks(b, b->max_bpc_f), s);
        } else {
          BatchArgs<float> a = make_args<float>(b);
          a.N = steps; a.K = steps; a.nseg = 1; a.mode = 0;
          (void)hipEventRecord(e0, s);
          mrt::launch_batch_forward<float>(a, persistent_blocks(b, b->max_bpc_f), s);
        }
        rc = launch_error();
        (void)hipEventRecord(e1, s);
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = err(MRT_EHIP, "tuning sync failed");
        if (!rc) (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < ms_best) ms_best = ms;
      }
      if (rc) break;
      const double per = ms_best / steps;
      if (per < best_ms) {
        best_ms = per;
        best_w = w;
        best_b = bpc;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = build_tiles(b, best_w);
  if (rc) return rc;
  b->bpc = best_b;
  // the tuning passes ran the real kernels on the batch buffers: the barrier
  // must not have tripped
  unsigned* ab = reinterpret_cast<unsigned*>(b->host);
  HIP_OK(hipMemcpy(ab, &b->barrier->abort.v, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (*ab) return err(MRT_EHIP, "grid barrier timed out during tuning");
  if (best) {
    best->tile_w = best_w;
    best->blocks_per_cu = best_b;
    best->max_blocks_per_cu = maxb;
    best->ms_per_step = best_ms;
  }
  return MRT_OK;
}

int mrt_batch_set_timeout(mrt_batch* b, double seconds) {
  if (!b || !(seconds >= 0.0)) return err(MRT_EINVAL, "invalid timeout");
  b->timeout = (unsigned long long)(seconds * 1e3 * double(b->clock_khz));
  b->graph_valid = false;
  return MRT_OK;
}

int mrt_batch_iteration(mrt_batch* b, double zeta, int32_t use_graph,
                        void* stream) {
  if (!b) return err(MRT_EINVAL, "batch is NULL");
  if (std::isnan(zeta)) return err(MRT_EINVAL, "zeta is NaN");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return err(MRT_ESTATE, "batch belongs to another device");
  if (b->mode == 0) return err(MRT_ESTATE, "batch was created for forward solves only");
  hipStream_t cs = static_cast<hipStream_t>(stream);
  if (!use_graph) {
    int rc = enqueue(b, zeta, cs);
    if (!rc) b->iterated = true;
    return rc;
  }
  if (!b->graph_valid || b->graph_zeta != zeta) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    HIP_OK(hipStreamBeginCapture(b->ps, hipStreamCaptureModeThreadLocal));
    int rc = enqueue(b, zeta, b->ps);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->ps, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess)
      return err(MRT_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    b->graph = g;
    HIP_OK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_valid = true;
    b->graph_zeta = zeta;
  }
  HIP_OK(hipEventRecord(b->ev_in, cs));
  HIP_OK(hipStreamWaitEvent(b->ps, b->ev_in, 0));
  HIP_OK(hipGraphLaunch(b->exec, b->ps));
  HIP_OK(hipEventRecord(b->ev_out, b->ps));
  HIP_OK(hipStreamWaitEvent(cs, b->ev_out, 0));
  b->iterated = true;
  return MRT_OK;
}

int mrt_batch_forward(mrt_batch* b, void* stream) {
  if (!b) return err(MRT_EINVAL, "batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int bf = persistent_blocks(b, b->max_bpc_f);
  const int bs = std::min(b->ntiles, 4096);
  if (b->dtype == MRT_F64) {
    BatchArgs<double> a = make_args<double>(b);
    a.mode = 0; a.K = a.N; a.nseg = 1;
    mrt::launch_batch_forward<double>(a, bf, s);
    mrt::launch_batch_finalize<double>(a, static_cast<const double*>(b->buf[(b->N - 1) & 1]), bs, s);
  } else {
    BatchArgs<float> a = make_args<float>(b);
    a.mode = 0; a.K = a.N; a.nseg = 1;
    mrt::launch_batch_forward<float>(a, bf, s);
    mrt::launch_batch_finalize<float>(a, static_cast<const float*>(b->buf[(b->N - 1) & 1]), bs, s);
  }
  int rc = launch_error();
  if (rc) return rc;
  // a barrier that timed out leaves u(T) unwritten: report it here, since
  // no later call of the forward-only path reads the flag
  unsigned* ab =
      reinterpret_cast<unsigned*>(b->host + 2 * size_t(b->count) * mrt::kBatchSlots);
  HIP_OK(hipMemcpyAsync(ab, &b->barrier->abort.v, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (*ab) return err(MRT_EHIP, "grid barrier timed out: work-groups were not all resident");
  return MRT_OK;
}

int mrt_batch_scalars(mrt_batch* b, mrt_scalars* out, double* zeta_used,
                      void* stream) {
  if (!b || !out) return err(MRT_EINVAL, "NULL argument");
  if (!b->iterated) return err(MRT_ESTATE, "no iteration has run on the current control");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = size_t(b->count) * mrt::kBatchSlots;
  HIP_OK(hipMemcpyAsync(b->host, b->res_cost, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(b->host + n, b->res_grad, n * sizeof(double), hipMemcpyDeviceToHost, s));
  unsigned* ab = reinterpret_cast<unsigned*>(b->host + 2 * n);
  HIP_OK(hipMemcpyAsync(ab, &b->barrier->abort.v, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (*ab)
    return err(MRT_EHIP, "grid barrier timed out: work-groups were not all resident");
  bool finite = true;
  for (int k = 0; k < b->count; ++k) {
    const double* c = b->host + size_t(k) * mrt::kBatchSlots;
    const double* g = b->host + n + size_t(k) * mrt::kBatchSlots;
    out[k].J_track = c[0];
    out[k].J_reg = c[1];
    out[k].J = c[0] + c[1];
    out[k].grad_l2 = std::sqrt(g[2]);
    out[k].grad_inf = g[3];
    out[k].n_fluid = int64_t(b->L[k]) * b->L[k];
    if (zeta_used) zeta_used[k] = g[5];
    if (c[4] != 0.0 || g[4] != 0.0 || !std::isfinite(out[k].J)) finite = false;
  }
  if (!finite) return err(MRT_ENONFINITE, "non-finite cost or gradient in the batch");
  return MRT_OK;
}

}  // extern "C"
