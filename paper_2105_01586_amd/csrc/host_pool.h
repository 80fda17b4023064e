// Host-side helpers of the library's builders (the quadtree mesh, the s-step
// plan). Plain C++, no device code.
//
// HostVec: a vector whose resize() leaves new elements uninitialised, so
// that a large array is first written (and its pages first touched) by the
// tasks that fill it, in parallel, instead of being zeroed by one thread
// beforehand; elements must be of trivial types.
//
// HostPool: a process-wide pool of host worker threads.
// run(ntasks, body) calls body(task, ntasks) once for every task in
// [0, ntasks): the calling thread and the parked workers take tasks from a
// shared counter, and run returns when every task has finished. Work is split
// into tasks by the caller, independently of how many threads execute them,
// so results never depend on the thread count. One caller uses the workers at
// a time: a call made while another is running (builder threads of the server
// building meshes side by side) runs its tasks on its own thread, and so does
// a call in a process forked from the one that started the workers (a fork
// copies no threads).
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <memory>
#include <unistd.h>
#include <new>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

namespace fi {

template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    static_assert(std::is_trivially_default_constructible<U>::value, "trivial types only");
    ::new ((void*)p) U;
  }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new ((void*)p) U(std::forward<Args>(args)...);
  }
};

template <class T>
using HostVec = std::vector<T, NoInit<T>>;

class HostPool {
 public:
  // The pool (created on first use: up to 16 threads with the caller, one
  // per hardware thread). It lives until the process ends.
  static HostPool& get() {
    static HostPool* pool = new HostPool(
        (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency())));
    return *pool;
  }

  int threads() const { return (int)workers_.size() + 1; }

  template <class F>
  void run(int64_t ntasks, F&& body) {
    if (ntasks <= 0) return;
    if (ntasks == 1 || workers_.empty() || getpid() != pid_) {
      for (int64_t t = 0; t < ntasks; ++t) body(t, ntasks);
      return;
    }
    std::unique_lock<std::mutex> own(run_mu_, std::try_to_lock);
    if (!own.owns_lock()) {
      for (int64_t t = 0; t < ntasks; ++t) body(t, ntasks);
      return;
    }
    std::function<void(int64_t, int64_t)> job = [&body](int64_t t, int64_t nt) { body(t, nt); };
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &job;
      ntasks_ = ntasks;
      next_.store(0, std::memory_order_relaxed);
      busy_ = (int)workers_.size();
      ++gen_;
    }
    cv_.notify_all();
    take_tasks(job, ntasks);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return busy_ == 0; });
    job_ = nullptr;
  }

 private:
  explicit HostPool(int nthreads) : pid_(getpid()) {
    for (int i = 1; i < nthreads; ++i) workers_.emplace_back([this] { loop(); });
    for (auto& w : workers_) w.detach();  // parked until the process ends
  }

  void take_tasks(const std::function<void(int64_t, int64_t)>& job, int64_t nt) {
    for (int64_t t; (t = next_.fetch_add(1, std::memory_order_relaxed)) < nt;) job(t, nt);
  }

  void loop() {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int64_t, int64_t)>* job;
      int64_t nt;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        job = job_;
        nt = ntasks_;
      }
      take_tasks(*job, nt);
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (--busy_ == 0) done_cv_.notify_one();
      }
    }
  }

  const pid_t pid_;  // the process the workers run in
  std::vector<std::thread> workers_;
  std::mutex run_mu_;  // held by the caller that has the workers
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int64_t, int64_t)>* job_ = nullptr;
  int64_t ntasks_ = 0;
  std::atomic<int64_t> next_{0};
  int busy_ = 0;
  uint64_t gen_ = 0;
};

// Runs body(task, ntasks) for every task on the pool.
template <class F>
inline void pool_run(int64_t ntasks, F&& body) {
  HostPool::get().run(ntasks, std::forward<F>(body));
}

// Splits [0, n) into `parts` contiguous ranges; range t is [lo, hi).
inline std::pair<int64_t, int64_t> split_range(int64_t n, int64_t parts, int64_t t) {
  return {n * t / parts, n * (t + 1) / parts};
}

}  // namespace fi
