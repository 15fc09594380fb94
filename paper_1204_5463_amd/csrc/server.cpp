// Serving loop: continuous batching of solve requests (see dwsap.h).
//
// Requests wait in a FIFO queue. A slot admits the head of the queue as soon
// as the request's device-memory footprint fits the budget beside the
// requests already running; the slot then imports the gauge field and runs
// the lock-step FGMRES-DR solve on its own HIP stream, so admitted requests
// overlap on the device. Server allocations are stream-ordered
// (hipMallocAsync / hipFreeAsync on the slot's stream).
#include <string.h>

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dw_internal.hpp"

namespace dw {
size_t solver_bytes(long long sites, int m, int prec, int flags, int nrhs);
dw_status field_reload(dw_field f, const double* U_dev, double csw, hipStream_t stream);
}

using namespace dw;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device memory of the server's requests: a caching allocator shared by the
// slots. A block freed on a slot's stream waits in that stream's pending list
// until the slot has synchronised its stream (at the end of each request and
// after dropping a field); it then joins the free list, from which any slot
// takes it again when its size fits (at most a quarter larger). Requests of
// one lattice and RHS count therefore run on the same blocks, mapped once
// (allocating and freeing them through the driver or the stream-ordered pool
// for every request fragments the device memory: later requests ran up to
// three times slower). When the device has no room for a new block, the free
// blocks are released first. The admission budget counts only the requests'
// own footprints; free cached blocks are released on demand.
struct BlockCache {
  struct Block {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::mutex mu;
  std::vector<Block> free_blocks;
  std::unordered_map<void*, size_t> live;
  std::unordered_map<hipStream_t, std::vector<Block>> pending;

  void release_free() {  // with mu held
    for (auto& b : free_blocks) (void)hipFree(b.p);
    free_blocks.clear();
  }
  void* alloc(size_t bytes, hipStream_t s) {
    void* p = try_alloc(bytes);
    if (p) return p;
    // no room: the blocks this stream freed are reusable once it has drained
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
        hipStreamSynchronize(s) == hipSuccess) {
      retire(s);
      std::lock_guard<std::mutex> lk(mu);
      release_free();
    }
    (void)hipGetLastError();
    return try_alloc(bytes);
  }
  void* try_alloc(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    size_t best = SIZE_MAX;
    int pick = -1;
    for (int i = 0; i < (int)free_blocks.size(); ++i) {
      const Block& b = free_blocks[i];
      if (b.bytes >= bytes && b.bytes - bytes <= bytes / 4 && b.bytes < best) {
        best = b.bytes;
        pick = i;
      }
    }
    if (pick >= 0) {
      const Block b = free_blocks[pick];
      free_blocks.erase(free_blocks.begin() + pick);
      live[b.p] = b.bytes;
      return b.p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      release_free();
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    live[p] = bytes;
    return p;
  }
  void free(void* p, hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = live.find(p);
    if (it == live.end()) return;
    pending[s].push_back(Block{p, it->second});
    live.erase(it);
  }
  // the stream s has been synchronised: its freed blocks are reusable
  void retire(hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = pending.find(s);
    if (it == pending.end()) return;
    free_blocks.insert(free_blocks.end(), it->second.begin(), it->second.end());
    pending.erase(it);
  }
  ~BlockCache() {
    for (auto& b : free_blocks) (void)hipFree(b.p);
    for (auto& kv : pending)
      for (auto& b : kv.second) (void)hipFree(b.p);
    for (auto& kv : live) (void)hipFree(kv.first);
  }
};

void* cache_alloc(size_t bytes, hipStream_t s, void* user) { return static_cast<BlockCache*>(user)->alloc(bytes, s); }
void cache_free(void* p, hipStream_t s, void* user) { static_cast<BlockCache*>(user)->free(p, s); }

struct Req {
  uint64_t ticket = 0;
  dw_request r{};
  size_t footprint = 0;
  dw_req_state state = DW_REQ_QUEUED;
  std::vector<dw_solve_stats> stats;
  std::string err;
  double t_submit = 0, t_start = 0, t_end = 0;
};

}  // namespace

struct dw_server_s {
  dw_ctx user_ctx = nullptr;
  dw_ctx ictx = nullptr;  // allocates through `blocks`
  std::unique_ptr<BlockCache> blocks;
  dw_server_params p{};
  double budget = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Req>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
  double in_use = 0;
  bool stop = false;
  uint64_t next = 1;
  std::vector<std::thread> workers;
};

namespace {

// A slot keeps the field of its last request (its link copies, and with
// them the solver's workspace and captured restart cycles) while the next
// request it takes has the same lattice, block and clover presence: the new
// links are loaded into the same buffers and the captured cycles are
// replayed (the solver keeps them for equal parameters and RHS count).
// Otherwise, and whenever the slot goes idle, the field is freed. While the
// slot holds the field between requests, the footprint of the request that
// made it stays charged to the budget, so the other slots never count on
// that memory; the slot's next request takes the charge over.
struct SlotField {
  dw_field f = nullptr;
  int L[4] = {}, block[4] = {};
  bool clover = false;
  bool matches(const dw_request& r) const {
    if (!f || (r.csw != 0.0) != clover) return false;
    for (int i = 0; i < 4; ++i)
      if (L[i] != r.L[i] || block[i] != r.block[i]) return false;
    return true;
  }
  void drop(hipStream_t st, BlockCache* blocks) {
    if (!f) return;
    (void)hipStreamSynchronize(st);
    dw_field_destroy(f);
    f = nullptr;
    (void)hipStreamSynchronize(st);
    blocks->retire(st);
  }
};

void worker(dw_server s) {
  (void)hipSetDevice(s->ictx->device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  SlotField held;
  double held_fp = 0;  // footprint still charged for the held field
  auto release_held = [&]() {
    held.drop(st, s->blocks.get());
    std::lock_guard<std::mutex> lk(s->mu);
    s->in_use -= held_fp;
    held_fp = 0;
    s->cv.notify_all();
  };
  while (true) {
    std::shared_ptr<Req> rq;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // Admission in arrival order with backfilling: the head runs once its
      // footprint fits beside the running requests; a later request may
      // run before it only if the memory the head needs stays free, so
      // backfilled requests never delay the head's admission for memory.
      // The head always fits once none run (submit checked it against the
      // whole budget), so the queue drains, also after stop.
      // This slot's own held charge counts as free for its next request
      // (the held field is reused or freed before anything new is made).
      size_t pick = 0;
      auto admissible = [&]() {
        if (s->queue.empty()) return false;
        const double used = s->in_use - held_fp;
        const double head = (double)s->queue.front()->footprint;
        if (used + head <= s->budget) {
          pick = 0;
          return true;
        }
        for (size_t i = 1; i < s->queue.size(); ++i)
          if (used + head + (double)s->queue[i]->footprint <= s->budget) {
            pick = i;
            return true;
          }
        return false;
      };
      if (!admissible() && held.f) {
        // going idle: give the held field (and its charge) back before waiting
        lk.unlock();
        release_held();
        lk.lock();
      }
      s->cv.wait(lk, [&] { return admissible() || (s->stop && s->queue.empty()); });
      if (s->queue.empty()) break;
      rq = s->queue[pick];
      s->queue.erase(s->queue.begin() + (long)pick);
      s->in_use += (double)rq->footprint - held_fp;
      held_fp = 0;
      rq->state = DW_REQ_RUNNING;
      rq->t_start = now_s();
    }
    dw_status status = have_stream ? DW_OK : DW_EHIP;
    std::string err = have_stream ? "" : "could not create a stream for the server slot";
    if (status == DW_OK) {
      if (held.matches(rq->r)) {
        status = field_reload(held.f, rq->r.U, rq->r.csw, st);
        if (status != DW_OK) {
          err = dw_last_error();
          held.drop(st, s->blocks.get());
        }
      } else {
        held.drop(st, s->blocks.get());
        dw_field f = nullptr;
        status = dw_field_create(s->ictx, rq->r.L, rq->r.block, rq->r.U, st, &f);
        if (status == DW_OK && rq->r.csw != 0.0) {
          status = dw_field_set_clover(f, rq->r.csw, st);
          if (status != DW_OK) {
            err = dw_last_error();
            dw_field_destroy(f);
            f = nullptr;
          }
        } else if (status != DW_OK) {
          err = dw_last_error();
        }
        if (status == DW_OK) {
          f->memory_reserved = true;  // the footprint charged covers the whole request
          held.f = f;
          for (int i = 0; i < 4; ++i) {
            held.L[i] = rq->r.L[i];
            held.block[i] = rq->r.block[i];
          }
          held.clover = rq->r.csw != 0.0;
        }
      }
      if (status == DW_OK) {
        // every request runs on captured restart cycles
        fgmresdr_params prm = rq->r.params;
        prm.flags |= DW_SOLVE_GRAPHS;
        status = fgmresdr_solve(held.f, rq->r.m0, &prm, rq->r.b, rq->r.x, rq->r.nrhs, rq->stats.data(), st);
        if (status != DW_OK && status != DW_ENOTCONV) {
          err = dw_last_error();
          held.drop(st, s->blocks.get());
        }
      }
      (void)hipStreamSynchronize(st);
      s->blocks->retire(st);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      // a field kept for the next request keeps its charge
      if (held.f) held_fp = (double)rq->footprint;
      else s->in_use -= (double)rq->footprint;
      rq->t_end = now_s();
      rq->state = (status == DW_OK || status == DW_ENOTCONV) ? DW_REQ_DONE : DW_REQ_FAILED;
      rq->err = err;
    }
    s->cv.notify_all();
  }
  release_held();
  if (have_stream) (void)hipStreamDestroy(st);
}

bool valid_geom(const dw_request* q, Geom* g) {
  int L[4] = {q->L[0], q->L[1], q->L[2], q->L[3]}, B[4] = {q->block[0], q->block[1], q->block[2], q->block[3]};
  return make_geom(L, B, g) == nullptr;
}

}  // namespace

extern "C" {

size_t dw_request_footprint(const dw_request* q) {
  Geom g;
  if (!q || q->nrhs < 1 || !valid_geom(q, &g)) return 0;
  const int prec = q->params.sap.storage;
  if (prec < 0 || prec > 3 || q->params.m < 1 || q->params.m > 48) return 0;
  const size_t links = (size_t)g.V * 36 * (16 + 8 + 4 + 4) * (q->csw != 0.0 ? 2 : 1);  // + clover copies
  return links + solver_bytes(g.V, q->params.m, prec, q->params.flags, q->nrhs);
}

dw_status dw_server_create(dw_ctx ctx, const dw_server_params* p, dw_server* out) {
  clear_error();
  if (!ctx || !p || !out || p->slots < 1 || p->queue_capacity < 1 || p->budget_bytes < 0) {
    set_error("dw_server_create: invalid argument");
    return DW_EINVAL;
  }
  *out = nullptr;
  DW_CHECK_HIP(hipSetDevice(ctx->device));
  auto blocks = std::make_unique<BlockCache>();
  dw_allocator a{cache_alloc, cache_free, blocks.get()};
  dw_ctx ictx = nullptr;
  DW_TRY(dw_ctx_create(ctx->device, &a, &ictx));
  dw_server s = new dw_server_s;
  s->user_ctx = ctx;
  s->ictx = ictx;
  s->blocks = std::move(blocks);
  s->p = *p;
  if (p->budget_bytes > 0) {
    s->budget = p->budget_bytes;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      dw_ctx_destroy(ictx);
      delete s;
      set_error("dw_server_create: hipMemGetInfo failed");
      return DW_EHIP;
    }
    s->budget = 0.8 * (double)fr;
  }
  for (int i = 0; i < p->slots; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return DW_OK;
}

dw_status dw_server_destroy(dw_server s) {
  clear_error();
  if (!s) return DW_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  (void)hipDeviceSynchronize();
  dw_ctx_destroy(s->ictx);
  delete s;  // frees the cached blocks after the context (whose last frees return blocks to it)
  return DW_OK;
}

dw_status solve_submit(dw_server s, const dw_request* q, uint64_t* ticket) {
  clear_error();
  if (!s || !q || !ticket || !q->U || !q->b || !q->x || q->nrhs < 1 || !std::isfinite(q->csw)) {
    set_error("solve_submit: invalid argument");
    return DW_EINVAL;
  }
  Geom g;
  if (!valid_geom(q, &g)) {
    set_error("solve_submit: invalid lattice / block geometry");
    return DW_EINVAL;
  }
  for (int mu = 0; mu < 4; ++mu)
    if (q->params.sap.block[mu] != q->block[mu]) {
      set_error("solve_submit: params.sap.block differs from the request's block");
      return DW_EINVAL;
    }
  const fgmresdr_params& P = q->params;
  if (P.m < 1 || P.m > 48 || P.k < 0 || P.k >= P.m || P.k > 23 || P.max_iter < 1 || !(P.tol > 0) ||
      !(P.restart_t > 0) || P.sap.ncycles < 1 || P.sap.nmr < 0 || P.sap.storage < 0 || P.sap.storage > 3) {
    set_error("solve_submit: invalid solver parameters");
    return DW_EINVAL;
  }
  const size_t fp = dw_request_footprint(q);
  auto rq = std::make_shared<Req>();
  rq->r = *q;
  rq->footprint = fp;
  rq->stats.resize(q->nrhs);
  rq->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((double)fp > s->budget) {
      set_error("solve_submit: request needs %zu bytes, above the server budget %.0f", fp, s->budget);
      return DW_EINVAL;
    }
    if ((int)s->queue.size() >= s->p.queue_capacity) {
      set_error("solve_submit: queue full (%d requests)", s->p.queue_capacity);
      return DW_EBUSY;
    }
    rq->ticket = s->next++;
    s->queue.push_back(rq);
    s->reqs[rq->ticket] = rq;
    *ticket = rq->ticket;
  }
  s->cv.notify_all();
  return DW_OK;
}

dw_status solve_poll(dw_server s, uint64_t ticket, dw_req_state* state, dw_solve_stats* stats,
                     dw_request_times* times) {
  clear_error();
  if (!s || !state) {
    set_error("solve_poll: invalid argument");
    return DW_EINVAL;
  }
  std::shared_ptr<Req> rq;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
      set_error("solve_poll: unknown ticket %llu", (unsigned long long)ticket);
      return DW_ENOTFOUND;
    }
    rq = it->second;
    *state = rq->state;
    if (rq->state == DW_REQ_DONE || rq->state == DW_REQ_FAILED) s->reqs.erase(it);
  }
  if (*state == DW_REQ_DONE || *state == DW_REQ_FAILED) {
    if (stats) memcpy(stats, rq->stats.data(), rq->stats.size() * sizeof(dw_solve_stats));
    if (times) {
      times->queued = rq->t_start - rq->t_submit;
      times->running = rq->t_end - rq->t_start;
      times->latency = rq->t_end - rq->t_submit;
    }
    if (*state == DW_REQ_FAILED) set_error("%s", rq->err.c_str());
  }
  return DW_OK;
}

}  // extern "C"
