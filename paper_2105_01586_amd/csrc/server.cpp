// Batched serving of inpainting + tonal-optimisation requests on one GPU.
//
// A request is an image with its mask; the server builds its mesh, computes
// the harmonic inpainting (Section 2.2) and then runs a fixed number of CGLS
// iterations of tonal optimisation (Section 4). Requests of any size and
// density share the GPU by continuous batching:
//
//   builder threads  build the quadtree mesh on the host, reserve the
//                    request's device footprint in the arena (admission by
//                    HBM footprint: a request waits until its bound fits),
//                    upload and assemble it on their own stream;
//   the engine       keeps up to max_slots requests resident. Every solve of
//                    every resident request advances in the same step
//                    launches (one launch per CG step for all of them); when
//                    a request's solve ends, the engine queues the
//                    request's next non-solve kernels (interpolation,
//                    adjoint, CGLS updates) and starts its next solve, while
//                    the others keep stepping. Requests join and leave
//                    between chunks of step launches.
//
// The host stays two chunks ahead of the device and learns that a solve has
// ended from the state each step launch writes to pinned host memory. Each
// request's arithmetic is the same as that of the single-request calls
// (fi_inpaint, fi_tonal_opt), so a result does not depend on what else was
// in the batch.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "internal.h"

namespace fi {

// ------------------------------------------------------------------ arena --
int Arena::init(int device, size_t bytes) {
  (void)device;
  bytes &= ~(size_t)255;
  if (bytes == 0) return fail(FI_E_INVALID, "arena size is zero");
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? FI_E_NOMEM : FI_E_HIP,
                std::string("arena allocation failed: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(mu_);
  base_ = (char*)p;
  owned_ = true;
  cap_ = bytes;
  used_ = peak_ = 0;
  free_.clear();
  live_.clear();
  free_[0] = bytes;
  return FI_OK;
}

void Arena::init_view(void* base, size_t bytes) {
  std::lock_guard<std::mutex> lk(mu_);
  base_ = (char*)base;
  owned_ = false;
  cap_ = bytes & ~(size_t)255;
  used_ = peak_ = 0;
  free_.clear();
  live_.clear();
  if (cap_) free_[0] = cap_;
}

void Arena::release() {
  std::lock_guard<std::mutex> lk(mu_);
  if (base_ && owned_) (void)hipFree(base_);
  base_ = nullptr;
  owned_ = false;
  cap_ = used_ = 0;
  free_.clear();
  live_.clear();
}

void* Arena::alloc(size_t bytes) {
  bytes = std::max<size_t>(256, (bytes + 255) & ~(size_t)255);
  std::lock_guard<std::mutex> lk(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > bytes) free_[off + bytes] = len - bytes;
    live_[off] = bytes;
    used_ += bytes;
    peak_ = std::max(peak_, used_);
    return base_ + off;
  }
  return nullptr;
}

void Arena::free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  const size_t off = (size_t)((char*)p - base_);
  auto lv = live_.find(off);
  if (lv == live_.end()) return;
  size_t start = off, len = lv->second;
  used_ -= len;
  live_.erase(lv);
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == start + len) {  // merge with the next range
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // and with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == start) {
      start = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = len;
}

size_t Arena::used() const {
  std::lock_guard<std::mutex> lk(mu_);
  return used_;
}

size_t Arena::peak() const {
  std::lock_guard<std::mutex> lk(mu_);
  return peak_;
}

namespace {

// ------------------------------------------------------------- footprint --
// Upper bound of the device bytes a request takes: every allocation of the
// mesh, its matrices, the solver, the CGLS workspace and the request's own
// image and g, each rounded to 256 bytes. Matrix sizes use the vertex degree
// bound deg(v) <= incident triangles + 1.
int64_t footprint_bound(const HostMesh& H, int iters) {
  const int64_t V = H.V(), T = H.T(), L = H.L(), P = (int64_t)H.N * H.N;
  const int64_t m = (int64_t)H.mask_vids.size(), n = (int64_t)H.free_vids.size();
  // sum over the free (mask) vertices of incident triangles + 1
  int64_t deg_free = n, deg_mask = m;
  for (int64_t e = 0; e < 3 * T; ++e) {
    if (H.vmap[(size_t)H.tri[(size_t)e]] >= 0) ++deg_free;
    else ++deg_mask;
  }
  int64_t total = 0;
  auto add = [&](int64_t count, int64_t size) {
    int64_t b = std::max<int64_t>(count, 1) * size;
    total += std::max<int64_t>(256, (b + 255) & ~(int64_t)255);
  };
  // geometry
  add(2 * V, 4); add(3 * T, 4); add(4 * (L + 1), 4); add(V, 4); add(n, 4); add(m, 4); add(m, 4);
  add(V + 1, 4); add(3 * T, 4);
  // workspace
  add(std::max(2 * (n + 1), m + 1), 4); add(scan_tmp_ints(std::max({n, m, T, V}) + 1), 4);
  add(n + 1, 4); add(n + 1, 4); add(m + 1, 4);
  add(n, 8); add(n, 8); add(n, 4); add(n, 8); add(n, 8); add(n, 8); add(n, 8);
  add(n, 4); add(n, 4); add(4 * n, 4); add(4 * n, 4);
  add(n, 8); add(n, 8); add(4 * n, 8); add(4 * n, 8);
  add(kMaxGrid, 8); add(8, 8);
  add(V, 8); add(m, 8); add(3 * T, 8); add(m, 8); add((L + kBlock - 1) / kBlock, 8);
  add(P, 4); add(P, 4); add(T + 1, 4);  // owner map and per-triangle pixel lists
  // matrices
  add(deg_free, 4); add(deg_free, 8); add(deg_free, 4); add(deg_free, 4); add(deg_free, 8);
  add(deg_mask, 4); add(deg_mask, 8);
  // solver set-up
  const int64_t grid = ((n + kBatchBS - 1) / kBatchBS + 7) / 8 * 8;
  add(4, 4); add(4, 8); add(4 * kRedMaxBlocks, 8); add(8, 8); add(2, 96); add(2 * 4 * grid, 8);
  add((int64_t)kMaxEll * ((n + 63) / 64 * 64), 4);
  // CGLS workspace and the request's buffers
  add(m, 8); add(m, 8); add(P, 8); add(P, 8); add(n, 8); add(8, 8);
  add(P, 1); add(m, 8);
  // the S-iteration solver's plan and vectors, and the plan build's scratch
  total += ss_footprint(n);
  total += ss_plan_scratch_bound(n);
  (void)iters;
  return total;
}

double clock_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// --------------------------------------------------------------- requests --
struct Job {
  uint64_t ticket = 0;
  int side = 0;
  std::vector<uint8_t> f;
  std::vector<int32_t> mask;
  int iters = 0;
  double* g_out = nullptr;
  fi_solve_opts io{};

  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  fi_mesh* M = nullptr;
  uint8_t* d_f = nullptr;
  double* d_g = nullptr;
  double* h_out = nullptr;  // pinned: g (m), then the CGLS scalars (8)
  // The request's device memory: one contiguous region of the server's
  // arena, as large as the footprint bound, taken at admission; the mesh
  // and the request's buffers are carved out of it (sub), so a request never
  // waits for or fails on memory once admitted, whatever the arena's
  // fragmentation, and memory the solver allocates on first use is there.
  void* region = nullptr;
  std::unique_ptr<Arena> sub;
  Cgls c;
  int slot = -1;
  bool solving = false, advance = false, finished = false, done = false;
  bool collected = false, reaped = false;  // deleted once both hold
  int64_t armed_at = -1, finish_at = -1;
  int epoch = 0;  // the running solve's id in the mesh's host mirror
  int status = FI_OK;
  std::string error;
  int64_t inner_iterations = 0;
  int64_t device_bytes = 0, bound = 0;
  double mse_inpaint = 0, mse_tonal = 0;
};

}  // namespace
}  // namespace fi

struct fi_server {
  fi_server_opts opts{};
  int device = 0;
  bool batched = true;
  fi_ctx ctx_run, ctx_build;
  fi::Arena arena;
  double t0 = 0;

  std::mutex mu;
  std::condition_variable cv_build;  // builders: new requests, freed memory, shutdown
  std::condition_variable cv_engine; // engine: ready requests, shutdown
  std::condition_variable cv_done;   // pollers
  std::deque<fi::Job*> pending;      // submitted, not yet built
  std::deque<fi::Job*> ready;        // uploaded, waiting for a slot
  std::deque<fi::Job*> reap;         // finished: pinned buffers to free
  std::unordered_map<uint64_t, fi::Job*> jobs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int in_flight = 0;                 // submitted and not yet finished

  std::vector<std::thread> builders;
  std::thread engine;

  // engine state
  std::vector<fi::Job*> active;
  std::vector<int> free_slots;
  static constexpr int kRing = 4;
  hipEvent_t ev[kRing] = {};         // one per engine iteration, reused in turn
  fi_server_stats st{};
  std::string engine_error;
};

namespace fi {
namespace {

double since(const fi_server* S) { return clock_s() - S->t0; }

void finish_locked(fi_server* S, Job* J) {
  J->done = true;
  J->t_done = since(S);
  if (J->status == FI_OK) ++S->st.jobs_done;
  else ++S->st.jobs_failed;
  --S->in_flight;
  S->cv_done.notify_all();
  S->cv_engine.notify_all();
}

// Host-side release of a finished request (pinned memory, events); the
// device memory went back to the arena when the request finished.
void reap_job(fi_server* S, Job* R) {
  if (R->M) free_mesh(R->M);
  R->M = nullptr;
  if (R->h_out) (void)hipHostFree(R->h_out);
  R->h_out = nullptr;
  std::lock_guard<std::mutex> lk(S->mu);
  R->reaped = true;
  if (R->collected) delete R;
}

// ---------------------------------------------------------------- builders --
int build_job(fi_server* S, Job* J) {
  fi_host_mesh* hm = nullptr;
  int rc = fi_host_mesh_build(J->side, J->side, J->mask.data(), (int64_t)J->mask.size(), &hm);
  std::vector<int32_t>().swap(J->mask);
  if (rc) return rc;
  std::unique_ptr<fi_host_mesh, int (*)(fi_host_mesh*)> keep(hm, fi_host_mesh_destroy);
  const int64_t bound = footprint_bound(hm->mesh, J->iters);
  J->bound = bound;
  if (bound > (int64_t)S->arena.capacity())
    return fail(FI_E_NOMEM, "request needs more device memory than the server's budget");
  {  // admission: wait until a contiguous region of the bound is free
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_build.wait(lk, [&] { return (J->region = S->arena.alloc((size_t)bound)) != nullptr; });
  }
  J->sub.reset(new Arena());
  J->sub->init_view(J->region, ((size_t)bound + 255) & ~(size_t)255);
  fi_mesh* M = nullptr;
  hm = keep.release();
  rc = mesh_upload(&S->ctx_build, &hm, J->sub.get(), &M);
  if (hm) fi_host_mesh_destroy(hm);
  if (rc) return rc;
  J->M = M;
  J->c.M = M;
  rc = device_alloc(M, (void**)&J->d_f, (size_t)M->P);
  if (!rc) rc = device_alloc(M, (void**)&J->d_g, (size_t)std::max<int64_t>(M->m, 1) * 8);
  if (!rc) rc = J->c.alloc();
  if (!rc) {
    hipError_t e = hipMemcpyAsync(J->d_f, J->f.data(), (size_t)M->P, hipMemcpyHostToDevice,
                                  S->ctx_build.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->ctx_build.stream);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&J->h_out, (size_t)(M->m + 8) * sizeof(double),
                        hipHostMallocDefault);
    if (e != hipSuccess) rc = fail(FI_E_HIP, hipGetErrorString(e));
  }
  J->device_bytes = M->device_bytes;
  if (rc) return rc;
  std::vector<uint8_t>().swap(J->f);  // the image now lives on the device
  J->c.f = J->d_f;
  J->c.g = J->d_g;
  J->c.start_from_g = false;
  return FI_OK;
}

// Returns the request's region to the arena (callers notify the builders).
void release_job_memory(fi_server* S, Job* J) {
  if (J->M) J->M->allocations.clear();  // they lie in the region
  if (J->region) S->arena.free(J->region);
  J->region = nullptr;
}

void builder_main(fi_server* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    Job* J = nullptr;
    Job* R = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_build.wait(lk, [&] { return S->stopping || !S->pending.empty() || !S->reap.empty(); });
      if (!S->reap.empty()) {
        R = S->reap.front();
        S->reap.pop_front();
      } else if (!S->pending.empty()) {
        J = S->pending.front();
        S->pending.pop_front();
      } else if (S->stopping) {
        return;
      }
    }
    if (R) {
      reap_job(S, R);
      continue;
    }
    const int rc = build_job(S, J);
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc) {
      J->status = rc;
      J->error = fi_last_error();
      release_job_memory(S, J);
      S->reap.push_back(J);
      finish_locked(S, J);
      S->cv_build.notify_all();
      continue;
    }
    J->t_admit = since(S);
    S->ready.push_back(J);
    S->cv_engine.notify_all();
  }
}

// ------------------------------------------------------------------ engine --
Cgls::Seg next_seg(const Job* J) {
  switch (J->c.seg) {
    case Cgls::kInpaint: return J->iters > 0 ? Cgls::kAdjoint : Cgls::kDone;
    case Cgls::kAdjoint: return J->c.k < J->iters ? Cgls::kApplyP : Cgls::kFinal;
    case Cgls::kApplyP: return Cgls::kAdjoint;
    default: return Cgls::kDone;
  }
}

// Queues the copies of the results into the request's pinned buffer.
int queue_results(Job* J) {
  fi_mesh* M = J->M;
  FI_HIP_TRY(hipMemcpyAsync(J->h_out, J->d_g, (size_t)M->m * sizeof(double),
                            hipMemcpyDeviceToHost, M->ctx->stream));
  FI_HIP_TRY(hipMemcpyAsync(J->h_out + M->m, M->d_tsc, 8 * sizeof(double), hipMemcpyDeviceToHost,
                            M->ctx->stream));
  return FI_OK;
}

void collect_results(fi_server* S, Job* J) {
  fi_mesh* M = J->M;
  if (J->status == FI_OK) {
    const double* sc = J->h_out + M->m;
    J->mse_inpaint = sc[Cgls::kScRR0] / (double)M->P;
    J->mse_tonal = J->iters > 0 ? sc[Cgls::kScSSE] / (double)M->P : J->mse_inpaint;
    if (J->g_out) std::memcpy(J->g_out, J->h_out, (size_t)M->m * sizeof(double));
  }
  release_job_memory(S, J);
}

// Sequential mode: one request at a time, each solve on its own (FP64 or
// FP32 + refinement with the single-mesh solver).
int run_sequential(fi_server* S, Job* J) {
  fi_mesh* M = J->M;
  M->ctx = &S->ctx_run;
  J->c.seg = Cgls::kInpaint;
  for (;;) {
    int rc = J->c.pre();
    if (rc) return rc;
    fi_solve_stats st{};
    rc = solve_free(M, &J->io, &st, J->c.x0);
    J->inner_iterations += st.iterations;
    if (rc) return rc;
    if (st.status != FI_OK) return fail(FI_E_NO_CONVERGENCE, "inner solve did not converge");
    if ((rc = J->c.post())) return rc;
    const Cgls::Seg nx = next_seg(J);
    if (nx == Cgls::kDone) break;
    J->c.seg = nx;
  }
  int rc = queue_results(J);
  if (rc) return rc;
  FI_HIP_TRY(hipStreamSynchronize(S->ctx_run.stream));
  return FI_OK;
}

// Batched mode: start the current segment's solve of a resident request.
int start_segment(fi_server* S, Job* J, int64_t it) {
  int rc = J->c.pre();
  if (rc) return rc;
  if ((rc = solve_arm(J->M, &J->io, &J->epoch, J->c.x0))) return rc;
  J->solving = true;
  J->armed_at = it;
  (void)S;
  return FI_OK;
}

int advance(fi_server* S, Job* J, int64_t it) {
  int rc = J->c.post();
  if (rc) return rc;
  const Cgls::Seg nx = next_seg(J);
  if (nx == Cgls::kDone) {
    if ((rc = queue_results(J))) return rc;
    J->finished = true;
    J->finish_at = it;
    return FI_OK;
  }
  J->c.seg = nx;
  return start_segment(S, J, it);
}

void fail_job(Job* J, int rc, int64_t it) {
  J->status = rc;
  J->error = fi_last_error();
  J->solving = false;
  J->finished = true;
  J->finish_at = it;
}

void engine_batched(fi_server* S) {
  int64_t it = 0;
  const int chunk = S->opts.chunk;
  for (;;) {
    // admit ready requests into free slots
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->active.empty()) {
        S->cv_engine.wait(lk, [&] { return !S->ready.empty() || (S->stopping && S->in_flight == 0); });
        if (S->ready.empty()) return;
      }
      while (!S->ready.empty() && !S->free_slots.empty()) {
        Job* J = S->ready.front();
        S->ready.pop_front();
        J->slot = S->free_slots.back();
        S->free_slots.pop_back();
        J->M->ctx = &S->ctx_run;
        J->t_start = since(S);
        J->c.seg = Cgls::kInpaint;
        J->advance = false;
        S->active.push_back(J);
      }
      S->st.peak_resident = std::max<int64_t>(S->st.peak_resident, (int64_t)S->active.size());
    }
    // queue every request's next kernels
    for (Job* J : S->active) {
      if (J->finished) continue;
      int rc = FI_OK;
      if (J->armed_at < 0) rc = start_segment(S, J, it);
      else if (J->advance) {
        J->advance = false;
        rc = advance(S, J, it);
      }
      if (rc) fail_job(J, rc, it);
    }
    // one chunk of step launches over the requests that are solving
    std::vector<BatchSlot> act;
    for (Job* J : S->active)
      if (J->solving) act.push_back(BatchSlot{J->M});
    hipStream_t st = S->ctx_run.stream;
    int rc = FI_OK;
    if (!act.empty()) {
      rc = batch_launch_steps(st, act, chunk);
      S->st.step_rounds += chunk;
      S->st.slot_steps += (int64_t)chunk * (int64_t)act.size();
    }
    hipError_t e = hipSuccess;
    if (!rc) e = hipEventRecord(S->ev[it % fi_server::kRing], st);
    if (rc || e != hipSuccess) {  // the stream is unusable: fail everything resident
      S->engine_error = rc ? fi_last_error() : hipGetErrorString(e);
      (void)hipStreamSynchronize(st);
      std::lock_guard<std::mutex> lk(S->mu);
      for (Job* J : S->active) {
        J->status = FI_E_HIP;
        J->error = S->engine_error;
        release_job_memory(S, J);
        S->free_slots.push_back(J->slot);
        S->reap.push_back(J);
        finish_locked(S, J);
      }
      S->active.clear();
      S->cv_build.notify_all();
      ++it;
      continue;
    }
    // Pace the host two iterations ahead of the device; everything queued up
    // to iteration `done_it` has then finished.
    int64_t done_it = -1;
    if (it >= 2) {
      (void)hipEventSynchronize(S->ev[(it - 2) % fi_server::kRing]);
      done_it = it - 2;
    }
    {
      std::vector<Job*> keep;
      bool freed = false;
      for (Job* J : S->active) {
        if (J->finished && J->finish_at <= done_it) {
          collect_results(S, J);
          std::lock_guard<std::mutex> lk(S->mu);
          S->free_slots.push_back(J->slot);
          S->reap.push_back(J);
          finish_locked(S, J);
          freed = true;
          continue;
        }
        if (J->solving) {  // the solve reports its end through the host mirror
          fi_solve_stats ss{};
          int done = 0;
          int prc = solve_poll(J->M, J->epoch, &ss, &done);
          if (done) {
            J->solving = false;
            J->inner_iterations += ss.iterations;
            if (prc == FI_OK && ss.status != FI_OK)
              prc = fail(FI_E_NO_CONVERGENCE, "inner solve did not converge");
            if (prc) fail_job(J, prc, it);
            else J->advance = true;
          }
        }
        keep.push_back(J);
      }
      S->active.swap(keep);
      if (freed) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cv_build.notify_all();
      }
    }
    ++it;
  }
}

void engine_sequential(fi_server* S) {
  for (;;) {
    Job* J = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_engine.wait(lk, [&] { return !S->ready.empty() || (S->stopping && S->in_flight == 0); });
      if (S->ready.empty()) return;
      J = S->ready.front();
      S->ready.pop_front();
      S->st.peak_resident = std::max<int64_t>(S->st.peak_resident, 1);
    }
    J->t_start = since(S);
    int rc = run_sequential(S, J);
    if (rc) {
      J->status = rc;
      J->error = fi_last_error();
      (void)hipStreamSynchronize(S->ctx_run.stream);
    }
    collect_results(S, J);
    std::lock_guard<std::mutex> lk(S->mu);
    S->reap.push_back(J);
    finish_locked(S, J);
    S->cv_build.notify_all();
  }
}

void engine_main(fi_server* S) {
  (void)hipSetDevice(S->device);
  if (S->batched) engine_batched(S);
  else engine_sequential(S);
}

void destroy_server(fi_server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_engine.notify_all();
  S->cv_build.notify_all();
  if (S->engine.joinable()) S->engine.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->cv_build.notify_all();
  }
  for (auto& t : S->builders)
    if (t.joinable()) t.join();
  std::deque<Job*> rest;
  rest.swap(S->reap);
  for (Job* R : rest) reap_job(S, R);
  // requests never collected (all reaped by now)
  for (auto& kv : S->jobs) delete kv.second;
  S->jobs.clear();
  if (S->ctx_run.stream) (void)hipStreamSynchronize(S->ctx_run.stream);
  for (int k = 0; k < fi_server::kRing; ++k)
    if (S->ev[k]) (void)hipEventDestroy(S->ev[k]);
  S->arena.release();
  if (S->ctx_run.stream) (void)hipStreamDestroy(S->ctx_run.stream);
  if (S->ctx_build.stream) (void)hipStreamDestroy(S->ctx_build.stream);
  delete S;
}

}  // namespace
}  // namespace fi

using namespace fi;

extern "C" {

void fi_server_opts_default(fi_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_slots = 16;
  o->precision = FI_PREC_FP32_IR;
  o->hbm_budget = (size_t)32 << 30;
  o->build_threads = 4;
  o->chunk = 8;
}

int fi_server_create(fi_ctx* ctx, const fi_server_opts* opts, fi_server** out) {
  if (!ctx || !out) return fail(FI_E_INVALID, "ctx or out is NULL");
  *out = nullptr;
  fi_server_opts o;
  fi_server_opts_default(&o);
  if (opts) o = *opts;
  if (o.max_slots < 1 || o.max_slots > kMaxSlots)
    return fail(FI_E_INVALID, "max_slots must be in 1..64");
  if (o.precision != FI_PREC_FP32_IR && o.precision != FI_PREC_FP64)
    return fail(FI_E_INVALID, "unknown precision");
  if (o.build_threads < 1 || o.build_threads > 64)
    return fail(FI_E_INVALID, "build_threads must be in 1..64");
  if (o.chunk < 2 || o.chunk > 256 || (o.chunk & 1)) return fail(FI_E_INVALID, "chunk must be even, 2..256");
  if (o.hbm_budget < ((size_t)1 << 20)) return fail(FI_E_INVALID, "hbm_budget below 1 MiB");
  FI_HIP_TRY(hipSetDevice(ctx->device));
  fi_server* S = new fi_server();
  S->opts = o;
  S->device = ctx->device;
  S->batched = o.precision == FI_PREC_FP32_IR && o.max_slots > 1;
  S->t0 = clock_s();
  S->ctx_run.device = S->ctx_build.device = ctx->device;
  auto bail = [&](int rc) {
    destroy_server(S);
    return rc;
  };
  hipError_t e = hipStreamCreateWithFlags(&S->ctx_run.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->ctx_build.stream, hipStreamNonBlocking);
  for (int k = 0; k < fi_server::kRing && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&S->ev[k], hipEventDisableTiming);
  if (e != hipSuccess) return bail(fail(FI_E_HIP, hipGetErrorString(e)));
  int rc = S->arena.init(ctx->device, o.hbm_budget);
  if (rc) return bail(rc);
  S->st.arena_bytes = (int64_t)S->arena.capacity();
  for (int s = o.max_slots - 1; s >= 0; --s) S->free_slots.push_back(s);
  for (int t = 0; t < o.build_threads; ++t) S->builders.emplace_back(builder_main, S);
  S->engine = std::thread(engine_main, S);
  *out = S;
  return FI_OK;
}

int fi_server_submit(fi_server* S, const fi_job_desc* d, uint64_t* ticket) {
  if (!S || !d || !ticket) return fail(FI_E_INVALID, "NULL argument");
  if (!d->f || (!d->mask && d->m > 0)) return fail(FI_E_INVALID, "f and mask are required");
  if (d->side < 2 || (d->side & (d->side - 1)) || d->side > 16384)
    return fail(FI_E_INVALID, "side must be a power of two in 2..16384");
  if (d->m < 1) return fail(FI_E_EMPTY_MASK, "empty mask: the problem is singular");
  if (d->tonal_iters < 0) return fail(FI_E_INVALID, "tonal_iters must be >= 0");
  const int64_t P = (int64_t)d->side * d->side;
  if (d->m > P) return fail(FI_E_INVALID, "mask larger than the image");
  for (int64_t i = 0; i < d->m; ++i)
    if (d->mask[i] < 0 || d->mask[i] >= P || (i && d->mask[i] <= d->mask[i - 1]))
      return fail(FI_E_INVALID, "mask must be strictly ascending pixel indices");
  Job* J = new Job();
  J->side = d->side;
  J->f.assign(d->f, d->f + P);
  J->mask.assign(d->mask, d->mask + d->m);
  J->iters = d->tonal_iters;
  J->g_out = d->g_out;
  fi_solve_opts io = resolve_opts(&d->inner);
  io.precision = S->opts.precision;
  J->io = io;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) {
    delete J;
    return fail(FI_E_INVALID, "server is shutting down");
  }
  J->ticket = S->next_ticket++;
  J->t_submit = since(S);
  S->jobs[J->ticket] = J;
  S->pending.push_back(J);
  ++S->in_flight;
  ++S->st.jobs_submitted;
  S->cv_build.notify_all();
  *ticket = J->ticket;
  return FI_OK;
}

int fi_server_poll(fi_server* S, uint64_t ticket, int wait, fi_job_result* res) {
  if (!S || !res) return fail(FI_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto f = S->jobs.find(ticket);
  if (f == S->jobs.end()) return fail(FI_E_INVALID, "unknown ticket");
  Job* J = f->second;
  if (wait) S->cv_done.wait(lk, [&] { return J->done; });
  std::memset(res, 0, sizeof(*res));
  res->done = J->done ? 1 : 0;
  if (!J->done) return FI_OK;
  res->status = J->status;
  res->mse_inpaint = J->mse_inpaint;
  res->mse_tonal = J->mse_tonal;
  res->inner_iterations = J->inner_iterations;
  res->t_submit = J->t_submit;
  res->t_admit = J->t_admit;
  res->t_start = J->t_start;
  res->t_done = J->t_done;
  res->device_bytes = J->device_bytes;
  res->footprint_bound = J->bound;
  std::snprintf(res->error, sizeof(res->error), "%s", J->error.c_str());
  // collected: deleted here or by the builder that releases its host side
  S->jobs.erase(f);
  J->collected = true;
  if (J->reaped) delete J;
  return FI_OK;
}

int fi_server_stats_get(fi_server* S, fi_server_stats* out) {
  if (!S || !out) return fail(FI_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->arena_peak_bytes = (int64_t)S->arena.peak();
  out->arena_used_bytes = (int64_t)S->arena.used();
  out->clock = since(S);
  return FI_OK;
}

double fi_server_clock(fi_server* S) { return S ? since(S) : 0.0; }

int fi_server_destroy(fi_server* S) {
  if (!S) return FI_OK;
  destroy_server(S);
  return FI_OK;
}

int fi_server_footprint(int side, const int32_t* mask, int64_t m, int tonal_iters,
                        int64_t* bytes) {
  if (!bytes) return fail(FI_E_INVALID, "bytes is NULL");
  fi_host_mesh* hm = nullptr;
  int rc = fi_host_mesh_build(side, side, mask, m, &hm);
  if (rc) return rc;
  *bytes = footprint_bound(hm->mesh, tonal_iters);
  fi_host_mesh_destroy(hm);
  return FI_OK;
}

}  // extern "C"
