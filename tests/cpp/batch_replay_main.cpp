// Stand-alone driver of the batched queue replay (cp_state_sim.cpp), built with the address
// and undefined-behaviour sanitizers by the tests.  Reads a descriptor file, writes one line
// per queue position and one per array.
//   input (little-endian): int64 count, int64 final_threshold, int64 hist_bits,
//   int64 side_bits, then count x {uint64 addr, int64 size, int64 k, int64 offset},
//   int64 total, then total float32 values.
//   output: "order j i" lines, then "array i status value less equal work_passes" lines.
#include <cstdio>
#include <vector>

#include "cp_state_sim.cpp"

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  int64_t hdr[4];
  if (std::fread(hdr, sizeof(int64_t), 4, f) != 4) return 4;
  const int64_t count = hdr[0];
  if (count < 1 || count > (1 << 20)) return 5;
  std::vector<uint64_t> addrs((size_t)count);
  std::vector<int64_t> sizes((size_t)count), ks((size_t)count), off((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    int64_t rec[4];
    if (std::fread(rec, sizeof(int64_t), 4, f) != 4) return 6;
    addrs[(size_t)i] = (uint64_t)rec[0];
    sizes[(size_t)i] = rec[1];
    ks[(size_t)i] = rec[2];
    off[(size_t)i] = rec[3];
  }
  int64_t total = 0;
  if (std::fread(&total, sizeof(int64_t), 1, f) != 1 || total < 0) return 7;
  std::vector<float> data((size_t)total + 1);
  if ((int64_t)std::fread(data.data(), sizeof(float), (size_t)total, f) != total) return 8;
  std::fclose(f);
  for (int64_t i = 0; i < count; ++i)  // every readable array must lie inside the data
    if (off[(size_t)i] >= 0 && sizes[(size_t)i] > 0 && off[(size_t)i] + sizes[(size_t)i] > total)
      return 9;
  std::vector<int64_t> order((size_t)count), less((size_t)count), equal((size_t)count);
  std::vector<int32_t> status((size_t)count), passes((size_t)count);
  std::vector<double> value((size_t)count);
  replay_batch_f32(data.data(), addrs.data(), off.data(), sizes.data(), ks.data(), count, hdr[1],
                   (int)hdr[2], (int)hdr[3], order.data(), status.data(), value.data(),
                   less.data(), equal.data(), passes.data());
  for (int64_t j = 0; j < count; ++j) std::printf("order %lld %lld\n", (long long)j, (long long)order[(size_t)j]);
  for (int64_t i = 0; i < count; ++i)
    std::printf("array %lld %d %.17g %lld %lld %d\n", (long long)i, status[(size_t)i],
                value[(size_t)i], (long long)less[(size_t)i], (long long)equal[(size_t)i],
                passes[(size_t)i]);
  return 0;
}
