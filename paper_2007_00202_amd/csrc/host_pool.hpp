// A small pool of host threads for independent per-job host work (the proxy
// sampling of a construction step).  parallel_for(n, fn) runs fn(i) for every
// i in [0, n) on the pool's threads and the caller and returns when all are
// done; the first exception is rethrown in the caller.  One parallel_for at a
// time: a caller that finds the pool busy (another handle's thread) runs its
// loop alone.
#pragma once
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace bfmf {

class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool;
    return pool;
  }

  void parallel_for(size_t n, const std::function<void(size_t)>& fn) {
    if (n == 0) return;
    std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
    if (n == 1 || workers_.empty() || !busy.owns_lock()) {
      for (size_t i = 0; i < n; ++i) fn(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_ = 0;
      active_ = workers_.size();
      err_ = nullptr;
      ++epoch_;
    }
    cv_.notify_all();
    work();  // the caller takes items too
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return active_ == 0; });
    fn_ = nullptr;
    if (err_) std::rethrow_exception(err_);
  }

  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++epoch_;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  HostPool() {
    unsigned hw = std::thread::hardware_concurrency();
    if (const char* e = std::getenv("BFMF_HOST_THREADS")) hw = (unsigned)std::max(1, std::atoi(e));
    const unsigned nthreads = std::min(15u, hw > 1 ? hw - 1 : 0u);
    for (unsigned t = 0; t < nthreads; ++t) workers_.emplace_back([this] { loop(); });
  }

  void work() {
    for (;;) {
      const size_t i = next_.fetch_add(1);
      if (i >= n_) break;
      try {
        (*fn_)(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu_);
        if (!err_) err_ = std::current_exception();
      }
    }
  }

  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || epoch_ != seen; });
        if (stop_) return;
        seen = epoch_;
      }
      work();
      std::lock_guard<std::mutex> lk(mu_);
      if (--active_ == 0) done_cv_.notify_all();
    }
  }

  std::vector<std::thread> workers_;
  std::mutex mu_, run_mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(size_t)>* fn_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0};
  size_t active_ = 0;
  uint64_t epoch_ = 0;
  bool stop_ = false;
  std::exception_ptr err_;
};

}  // namespace bfmf
