// Host worker threads for the library's setup work (partition, fills,
// packing, copies out of staging buffers).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <system_error>
#include <thread>
#include <vector>

namespace hm {

// Threads to use by default: the host's, at most 16.
inline int host_threads() { return (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

// Run `work` on the calling thread and on up to nt - 1 more threads, then
// join them all.  `work` must take its items from a shared counter, so that
// any number of threads finishes the job: a thread that cannot be started
// (the host is out of threads) only means fewer workers, never an exception
// unwinding past running threads.
template <class F>
void run_workers(int nt, F work) {
  std::vector<std::thread> th;
  for (int i = 1; i < nt; i++) {
    try {
      th.emplace_back(work);
    } catch (const std::system_error &) {
      break;
    } catch (const std::bad_alloc &) {
      break;
    }
  }
  work();
  for (auto &x : th) x.join();
}

// f(i) for every i in [0, count), items handed out one at a time to up to nt
// threads (f writes disjoint outputs).
template <class F>
void parallel_items(int64_t count, int nt, F f) {
  if (count <= 0) return;
  std::atomic<int64_t> next{0};
  run_workers((int)std::min<int64_t>(std::max(1, nt), count), [&]() {
    for (int64_t i; (i = next.fetch_add(1)) < count;) f(i);
  });
}

}  // namespace hm
