// Runs the library's host reference of the kd order (csrc/host.cpp) on keys
// read from a file and writes the order: the test pins the numpy rendering
// of the same order against it.  Input: int64 n, then n x 4 float32 keys.
// Output: n int32 segment numbers in kd order.
#include <cstdio>
#include <vector>

#include "../../paper_2112_10408_amd/csrc/host.h"

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  long long n = 0;
  if (std::fread(&n, sizeof(n), 1, f) != 1 || n < 0) return 4;
  std::vector<float> keys(4 * (size_t)n);
  if (std::fread(keys.data(), sizeof(float), keys.size(), f) != keys.size()) return 5;
  std::fclose(f);
  std::vector<int32_t> idx((size_t)n);
  for (long long i = 0; i < n; ++i) idx[(size_t)i] = (int32_t)i;
  tnn::host::kd_order(idx.data(), n, keys.data(), 64);
  FILE *o = std::fopen(argv[2], "wb");
  if (!o) return 6;
  if (std::fwrite(idx.data(), sizeof(int32_t), idx.size(), o) != idx.size()) return 7;
  std::fclose(o);
  return 0;
}
