// ORACLE DIRECTORY -- test and benchmark infrastructure only.
//
// The all-core CPU baseline the benchmark reports beside the single-threaded
// oracle: the same definition of the result (records ordered by their key
// bytes in memcmp order, equal keys in input order), computed by libstdc++'s
// parallel-mode stable sort over record indices on every host thread.  It
// shares no code with the GPU library.
#include <parallel/algorithm>

#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include <omp.h>

extern "C" {

// perm[k] = input index of output position k.  threads <= 0: all of them.
// Returns the number of threads used.
int oracle_parallel_sort_order(const uint8_t* in, uint64_t n, uint32_t rec, uint32_t key, uint64_t* perm,
                               int threads) {
  if (threads > 0) omp_set_num_threads(threads);
  const int used = omp_get_max_threads();
  std::iota(perm, perm + n, uint64_t{0});
  __gnu_parallel::stable_sort(perm, perm + n, [&](uint64_t a, uint64_t b) {
    return std::memcmp(in + a * rec, in + b * rec, key) < 0;
  });
  return used;
}

}  // extern "C"
