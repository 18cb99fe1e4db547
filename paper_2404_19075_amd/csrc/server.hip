// server.hip -- continuously batched queries of a trained field (the
// voxelisation / reprojection use of the network, Sec. IV).
//
// A server owns one HIP stream, the network's packed weights (resident for
// its lifetime) and a scheduler thread.  Requests are submitted from any
// thread and queue in arrival order.  The scheduler admits the queue's head
// whenever its output bytes fit in the memory budget and a descriptor slot is
// free, then repeatedly launches the query kernel over a tile table drawn
// round-robin from every admitted request: a request that arrives while
// others are on the GPU is admitted as soon as memory and a slot free up and
// its tiles share the very next launch with theirs.  Two launches are kept in
// flight; when one completes, the tiles it carried are credited and every
// request whose tiles are all done is completed (its output is then valid),
// its memory released.  Each tile's result depends only on its request and
// index, so a request's output is the same alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ctx.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  dinr_request r;
  float* out;
  uint64_t ticket;
  size_t bytes;
  int slot = -1;
  int64_t n_tiles = 0, issued = 0, finished = 0;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  int state = 0;  // 0 queued, 1 admitted, 2 done
};

struct Batch {
  hipEvent_t ev;
  QueryTile* h_tiles;  // pinned
  QueryTile* d_tiles;
  std::vector<std::pair<uint64_t, int64_t>> credit;  // (ticket, tiles in this batch)
  bool busy = false;
};

}  // namespace

struct dinr_server {
  dinr_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  const float* params = nullptr;
  void* Wpk = nullptr;
  void* WTpk = nullptr;
  float* bias = nullptr;
  float* wo = nullptr;
  PackArgs pk{};
  int max_active = 0;
  int max_tiles = 0;
  QueryDesc* d_desc = nullptr;
  QueryDesc* h_desc = nullptr;  // pinned staging of descriptors
  Batch batch[2];
  int next_batch = 0;
  size_t budget = 0, in_use = 0;
  std::mutex mu;
  std::condition_variable cv;   // work arrived / stop
  std::condition_variable done_cv;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> active;  // admission order
  std::vector<int> free_slots;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  int error = 0;
  std::thread th;
  int64_t launches = 0, tiles_run = 0;
};

static int tile_points(const dinr_ctx* c) { return c->tile; }

static int64_t tiles_of(const dinr_ctx* c, const dinr_request& r) {
  const int64_t n2 = (int64_t)r.n * r.n;
  const int T = tile_points(c);
  if (r.kind == DINR_QUERY_SLICE) return (n2 + T - 1) / T;
  const int rays_per_tile = T / r.samples_per_ray;
  return (n2 + rays_per_tile - 1) / rays_per_tile;
}

static void complete_batch(dinr_server* s, Batch& b) {
  // called with the lock held, after b.ev completed
  for (auto& cr : b.credit) {
    auto it = s->reqs.find(cr.first);
    if (it == s->reqs.end()) continue;
    Req& q = it->second;
    q.finished += cr.second;
    if (q.finished == q.n_tiles && q.state == 1) {
      q.state = 2;
      q.t_done = now_ms();
      s->in_use -= q.bytes;
      s->free_slots.push_back(q.slot);
      s->active.erase(std::find(s->active.begin(), s->active.end(), q.ticket));
    }
  }
  b.credit.clear();
  b.busy = false;
}

static void scheduler(dinr_server* s) {
  dinr_ctx* c = s->ctx;
  hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admit from the head of the queue while memory and slots allow
    while (!s->queue.empty() && !s->free_slots.empty()) {
      Req& q = s->reqs[s->queue.front()];
      if (s->in_use + q.bytes > s->budget) break;
      q.slot = s->free_slots.back();
      s->free_slots.pop_back();
      s->in_use += q.bytes;
      q.state = 1;
      q.t_admit = now_ms();
      QueryDesc d{};
      d.kind = q.r.kind;
      d.n = q.r.n;
      d.samples = q.r.kind == DINR_QUERY_SLICE ? 1 : q.r.samples_per_ray;
      const dinr_geometry& g = c->geom;
      d.tn = (float)(2.0 * (q.r.t - g.t0) / (g.t1 - g.t0) - 1.0);
      if (q.r.kind == DINR_QUERY_SLICE) {
        const double z0 = g.fov_kind == DINR_FOV_BOX ? g.fov[4] : g.fov[1];
        const double z1 = g.fov_kind == DINR_FOV_BOX ? g.fov[5] : g.fov[2];
        d.zn = (float)(2.0 * (q.r.z_or_theta - z0) / (z1 - z0) - 1.0);
      } else {
        d.cth = (float)std::cos(q.r.z_or_theta);
        d.sth = (float)std::sin(q.r.z_or_theta);
      }
      d.out = q.out;
      s->h_desc[q.slot] = d;
      // the descriptor reaches the device before any launch that uses it
      // (same stream); the pinned staging entry is not reused before the
      // slot is freed, i.e. after those launches completed
      hipMemcpyAsync(&s->d_desc[q.slot], &s->h_desc[q.slot], sizeof(QueryDesc),
                     hipMemcpyHostToDevice, s->st);
      s->active.push_back(q.ticket);
      s->queue.pop_front();
    }
    Batch& b = s->batch[s->next_batch];
    if (b.busy) {
      // wait for the older launch, then credit its tiles
      lk.unlock();
      hipEventSynchronize(b.ev);
      lk.lock();
      complete_batch(s, b);
      s->done_cv.notify_all();
      continue;
    }
    // build a launch: round-robin shares of the admitted requests' tiles
    int n = 0;
    int pending = 0;
    for (uint64_t t : s->active) {
      const Req& q = s->reqs[t];
      if (q.issued < q.n_tiles) ++pending;
    }
    if (pending > 0) {
      int left = s->max_tiles;
      for (int pass = 0; pass < 2 && left > 0; ++pass) {
        int want = 0;
        for (uint64_t t : s->active) {
          const Req& q = s->reqs[t];
          if (q.issued < q.n_tiles) ++want;
        }
        if (want == 0) break;
        const int share = std::max(1, left / want);
        for (uint64_t t : s->active) {
          Req& q = s->reqs[t];
          const int64_t k = std::min<int64_t>({(int64_t)share, q.n_tiles - q.issued, (int64_t)left});
          if (k <= 0) continue;
          for (int64_t i = 0; i < k; ++i) b.h_tiles[n + i] = QueryTile{q.slot, (int)(q.issued + i)};
          b.credit.emplace_back(q.ticket, k);
          q.issued += k;
          n += (int)k;
          left -= (int)k;
          if (left == 0) break;
        }
      }
    }
    if (n == 0) {
      // nothing to launch: finish the other launch if one is running, else sleep
      Batch& o = s->batch[s->next_batch ^ 1];
      if (o.busy) {
        lk.unlock();
        hipEventSynchronize(o.ev);
        lk.lock();
        complete_batch(s, o);
        s->done_cv.notify_all();
        continue;
      }
      if (s->stop) break;
      s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop && s->queue.empty()) break;
      continue;
    }
    hipMemcpyAsync(b.d_tiles, b.h_tiles, sizeof(QueryTile) * n, hipMemcpyHostToDevice, s->st);
    MlpArgs a{};
    a.Bmat = c->d_B;
    a.params = s->params;
    a.bo_off = c->bo_off;
    a.Wpk = s->Wpk;
    a.WTpk = s->WTpk;
    a.bias = s->bias;
    a.wo_perm = s->wo;
    for (int l = 0; l < c->L; ++l) {
      a.wpk_off[l] = s->pk.pk_off[l];
      a.wtpk_off[l] = s->pk.pkT_off[l];
    }
    a.wpk_bytes = s->pk.n_w * (int64_t)esize(c->prec);
    a.wtpk_bytes = s->pk.n_wt * (int64_t)esize(c->prec);
    a.L = c->L;
    a.out_act = c->mlp.out_act;
    a.act = c->mlp.act == DINR_SWISH ? 1 : 0;
    a.qdesc = s->d_desc;
    a.qtiles = b.d_tiles;
    a.n_qtiles = n;
    a.geom = c->gd;
    const int grid = std::min(n, c->n_cu);
    hipError_t e = launch_query(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, c->IN, c->H, a, grid,
                                s->st);
    if (e == hipSuccess) e = hipEventRecord(b.ev, s->st);
    if (e != hipSuccess) {
      s->error = DINR_EHIP;
      fail(c, DINR_EHIP, "query launch failed: %s", hipGetErrorString(e));
      b.credit.clear();
      s->stop = true;
      s->done_cv.notify_all();
      break;
    }
    b.busy = true;
    ++s->launches;
    s->tiles_run += n;
    s->next_batch ^= 1;
  }
  // drain: wait for launches still in flight
  for (auto& b : s->batch)
    if (b.busy) {
      lk.unlock();
      hipEventSynchronize(b.ev);
      lk.lock();
      complete_batch(s, b);
    }
  s->done_cv.notify_all();
}

extern "C" {

int dinr_server_create(dinr_ctx* c, const float* params_d, size_t budget, int32_t max_active,
                       dinr_server** out) {
  if (!out) return DINR_EINVAL;
  *out = nullptr;
  if (!c || !params_d) return DINR_EINVAL;
  if (max_active < 1 || max_active > 4096) return fail(c, DINR_EINVAL, "max_active in [1, 4096]");
  if (budget < 4096) return fail(c, DINR_ENOMEM, "server memory budget below 4 KiB");
  dinr_server* s = new dinr_server();
  s->ctx = c;
  s->params = params_d;
  s->budget = budget;
  s->max_active = max_active;
  s->max_tiles = 8 * c->n_cu;
  s->pk = pack_layout(c);
  bool ok = hipSetDevice(c->device) == hipSuccess &&
            hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc(&s->Wpk, s->pk.n_w * esize(c->prec)) == hipSuccess &&
            hipMalloc(&s->WTpk, std::max<int64_t>(s->pk.n_wt, 1) * esize(c->prec)) == hipSuccess &&
            hipMalloc(&s->bias, sizeof(float) * c->L * c->H) == hipSuccess &&
            hipMalloc(&s->wo, sizeof(float) * c->H) == hipSuccess &&
            hipMalloc(&s->d_desc, sizeof(QueryDesc) * max_active) == hipSuccess &&
            hipHostMalloc(&s->h_desc, sizeof(QueryDesc) * max_active, hipHostMallocDefault) ==
                hipSuccess;
  for (auto& b : s->batch) {
    ok = ok && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc(&b.h_tiles, sizeof(QueryTile) * s->max_tiles, hipHostMallocDefault) ==
             hipSuccess &&
         hipMalloc(&b.d_tiles, sizeof(QueryTile) * s->max_tiles) == hipSuccess;
  }
  if (ok) {
    ok = launch_pack(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, s->pk, params_d, s->Wpk, s->WTpk,
                     s->bias, s->wo, s->st) == hipSuccess &&
         hipStreamSynchronize(s->st) == hipSuccess;
  }
  if (!ok) {
    dinr_server_destroy(s);
    return fail(c, DINR_EHIP, "server resources could not be created");
  }
  for (int k = max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->th = std::thread(scheduler, s);
  *out = s;
  return DINR_OK;
}

int dinr_query(dinr_server* s, const dinr_request* r, float* out_d, uint64_t* ticket) {
  if (!s || !r || !out_d || !ticket) return DINR_EINVAL;
  dinr_ctx* c = s->ctx;
  if (r->kind != DINR_QUERY_SLICE && r->kind != DINR_QUERY_REPROJECTION)
    return fail(c, DINR_EINVAL, "request kind");
  if (r->n < 1 || r->n > 8192) return fail(c, DINR_EINVAL, "request size n in [1, 8192]");
  if (!std::isfinite(r->z_or_theta) || !std::isfinite(r->t)) return fail(c, DINR_EINVAL, "z/theta/t");
  if (r->kind == DINR_QUERY_REPROJECTION) {
    const int S = r->samples_per_ray;
    if (S < 1 || S > c->tile || c->tile % S != 0)
      return fail(c, DINR_EINVAL, "samples_per_ray must divide %d", c->tile);
  }
  const size_t bytes = sizeof(float) * (size_t)r->n * r->n;
  if (bytes > s->budget) return fail(c, DINR_ENOMEM, "request larger than the server budget");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop || s->error) return fail(c, DINR_EBUSY, "server stopped");
  Req q;
  q.r = *r;
  q.out = out_d;
  q.ticket = s->next_ticket++;
  q.bytes = bytes;
  q.n_tiles = tiles_of(c, *r);
  q.t_submit = now_ms();
  s->reqs.emplace(q.ticket, q);
  s->queue.push_back(q.ticket);
  *ticket = q.ticket;
  s->cv.notify_one();
  return DINR_OK;
}

int dinr_poll(dinr_server* s, uint64_t ticket, int32_t* done, double* latency_ms) {
  if (!s || !done) return DINR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(s->ctx, DINR_EINVAL, "unknown ticket");
  *done = it->second.state == 2 ? 1 : 0;
  if (latency_ms) *latency_ms = *done ? it->second.t_done - it->second.t_submit : -1.0;
  if (s->error) return s->error;
  return DINR_OK;
}

int dinr_query_wait(dinr_server* s, uint64_t ticket) {
  if (!s) return DINR_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(s->ctx, DINR_EINVAL, "unknown ticket");
  s->done_cv.wait(lk, [&] { return s->reqs[ticket].state == 2 || s->error || s->stop; });
  if (s->reqs[ticket].state == 2) return DINR_OK;
  return s->error ? s->error : DINR_EBUSY;
}

int dinr_query_release(dinr_server* s, uint64_t ticket) {
  if (!s) return DINR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state != 2) return DINR_EINVAL;
  s->reqs.erase(it);
  return DINR_OK;
}

int dinr_server_stats(dinr_server* s, int64_t* launches, int64_t* tiles, size_t* bytes_in_use,
                      int32_t* queued, int32_t* admitted) {
  if (!s) return DINR_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (launches) *launches = s->launches;
  if (tiles) *tiles = s->tiles_run;
  if (bytes_in_use) *bytes_in_use = s->in_use;
  if (queued) *queued = (int32_t)s->queue.size();
  if (admitted) *admitted = (int32_t)s->active.size();
  return DINR_OK;
}

int dinr_volume_write(dinr_server* s, const dinr_volume* v, const char* path,
                      dinr_volume_stats* stats) {
  if (!s) return DINR_EINVAL;
  dinr_ctx* c = s->ctx;
  if (!v || !path || !v->times) return fail(c, DINR_EINVAL, "null volume description");
  if (v->n < 1 || v->n > 8192 || v->nz < 1 || v->nt < 1 || v->slots < 0 || v->slots > 64)
    return fail(c, DINR_EINVAL, "volume: n in [1, 8192], nz, nt >= 1, slots in [0, 64]");
  for (int t = 0; t < v->nt; ++t)
    if (!std::isfinite(v->times[t])) return fail(c, DINR_EINVAL, "volume: non-finite time");
  const int slots = v->slots ? v->slots : 4;
  const int64_t n2 = (int64_t)v->n * v->n;
  const size_t bytes = (size_t)n2 * sizeof(float);
  if (bytes > s->budget) return fail(c, DINR_ENOMEM, "volume: a slice exceeds the server budget");
  const double t_start = now_ms();
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, DINR_EIO, "volume: cannot open %s", path);
  {
    char h[64] = {0};
    std::memcpy(h, "DINR4DV1", 8);
    const int64_t dims[4] = {v->nt, v->nz, v->n, v->n};
    std::memcpy(h + 8, dims, sizeof(dims));
    if (std::fwrite(h, 1, 64, f) != 64 ||
        std::fwrite(v->times, sizeof(double), (size_t)v->nt, f) != (size_t)v->nt) {
      std::fclose(f);
      return fail(c, DINR_EIO, "volume: header write failed");
    }
  }
  // slot buffers: the server writes dev[k]; the copy stream moves it to host[k]
  std::vector<float*> dev(slots, nullptr), host(slots, nullptr);
  std::vector<hipEvent_t> ev(slots, nullptr);
  hipStream_t cs = nullptr;
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
  for (int k = 0; k < slots && ok; ++k)
    ok = hipMalloc(&dev[k], bytes) == hipSuccess && hipHostMalloc(&host[k], bytes) == hipSuccess &&
         hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) == hipSuccess;
  int rc = ok ? DINR_OK : DINR_ENOMEM;
  // writer thread: slices leave in submission order
  std::mutex m;
  std::condition_variable cv;
  std::deque<int> ready;
  std::vector<char> is_free(slots, 1);
  bool quit = false, io_err = false;
  std::thread writer([&] {
    for (;;) {
      int k;
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return quit || !ready.empty(); });
        if (ready.empty()) return;
        k = ready.front();
        ready.pop_front();
      }
      bool bad = hipEventSynchronize(ev[k]) != hipSuccess;
      if (!bad) bad = std::fwrite(host[k], sizeof(float), (size_t)n2, f) != (size_t)n2;
      {
        std::lock_guard<std::mutex> lk(m);
        if (bad) io_err = true;
        is_free[k] = 1;
      }
      cv.notify_all();
    }
  });
  const GeomDev& g = c->gd;
  const double z0 = g.fov_kind == DINR_FOV_BOX ? c->geom.fov[4] : c->geom.fov[1];
  const double z1 = g.fov_kind == DINR_FOV_BOX ? c->geom.fov[5] : c->geom.fov[2];
  const int64_t total = (int64_t)v->nt * v->nz;
  std::deque<std::pair<int, uint64_t>> inflight;  // (slot, ticket), submission order
  int64_t next = 0;
  while (rc == DINR_OK && (next < total || !inflight.empty())) {
    while (rc == DINR_OK && next < total && (int)inflight.size() < slots) {
      int k = -1;
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] {
          return io_err || std::find(is_free.begin(), is_free.end(), 1) != is_free.end();
        });
        if (io_err) {
          rc = DINR_EIO;
          break;
        }
        k = (int)(std::find(is_free.begin(), is_free.end(), 1) - is_free.begin());
        is_free[k] = 0;
      }
      dinr_request r{};
      r.kind = DINR_QUERY_SLICE;
      r.n = v->n;
      const int64_t it = next / v->nz, kz = next % v->nz;
      r.z_or_theta = z0 + ((double)kz + 0.5) * (z1 - z0) / v->nz;
      r.t = v->times[it];
      uint64_t tk = 0;
      const int q = dinr_query(s, &r, dev[k], &tk);
      if (q != DINR_OK) {
        std::lock_guard<std::mutex> lk(m);
        is_free[k] = 1;
        rc = q;
        break;
      }
      inflight.emplace_back(k, tk);
      ++next;
    }
    if (rc != DINR_OK || inflight.empty()) break;
    const auto [k, tk] = inflight.front();
    inflight.pop_front();
    const int w = dinr_query_wait(s, tk);
    dinr_query_release(s, tk);
    if (w != DINR_OK) {
      rc = w;
      break;
    }
    if (hipMemcpyAsync(host[k], dev[k], bytes, hipMemcpyDeviceToHost, cs) != hipSuccess ||
        hipEventRecord(ev[k], cs) != hipSuccess) {
      rc = DINR_EHIP;
      break;
    }
    {
      std::lock_guard<std::mutex> lk(m);
      ready.push_back(k);
    }
    cv.notify_all();
  }
  // nothing may still write the slot buffers when they are freed
  for (const auto& q : inflight) {
    dinr_query_wait(s, q.second);
    dinr_query_release(s, q.second);
  }
  {
    std::lock_guard<std::mutex> lk(m);
    quit = true;
  }
  cv.notify_all();
  writer.join();
  if (rc == DINR_OK && io_err) rc = DINR_EIO;
  if (s->st) hipStreamSynchronize(s->st);
  if (cs) {
    hipStreamSynchronize(cs);
    hipStreamDestroy(cs);
  }
  for (int k = 0; k < slots; ++k) {
    if (ev[k]) hipEventDestroy(ev[k]);
    if (dev[k]) hipFree(dev[k]);
    if (host[k]) hipHostFree(host[k]);
  }
  const long end = std::ftell(f);
  if (std::fclose(f) != 0 && rc == DINR_OK) rc = DINR_EIO;
  if (stats) {
    stats->bytes = end;
    stats->seconds = (now_ms() - t_start) * 1e-3;
    stats->voxels_per_s = rc == DINR_OK ? (double)total * n2 / stats->seconds : 0.0;
  }
  if (rc == DINR_EIO) return fail(c, DINR_EIO, "volume: write to %s failed", path);
  if (rc == DINR_ENOMEM) return fail(c, DINR_ENOMEM, "volume: slot buffers");
  if (rc == DINR_EHIP) return fail(c, DINR_EHIP, "volume: device-to-host copy");
  return rc;
}

int dinr_server_destroy(dinr_server* s) {
  if (!s) return DINR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  if (s->st) hipStreamSynchronize(s->st);
  for (auto& b : s->batch) {
    if (b.ev) hipEventDestroy(b.ev);
    if (b.h_tiles) hipHostFree(b.h_tiles);
    if (b.d_tiles) hipFree(b.d_tiles);
  }
  hipFree(s->Wpk);
  hipFree(s->WTpk);
  hipFree(s->bias);
  hipFree(s->wo);
  hipFree(s->d_desc);
  if (s->h_desc) hipHostFree(s->h_desc);
  if (s->st) hipStreamDestroy(s->st);
  delete s;
  return DINR_OK;
}

}  // extern "C"
