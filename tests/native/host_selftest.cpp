// Self-test of the library's host-only logic (csrc/host.cpp), built with g++
// under the address and undefined-behaviour sanitizers by
// tests/test_sanitizers.py.  Exits 0 and prints "host ok" when every check
// holds; any sanitizer report aborts with a non-zero status.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <utility>
#include <vector>

#include "../../paper_2112_10408_amd/csrc/host.h"

using namespace tnn::host;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

static void offsets_and_counts() {
  const int64_t good[] = {0, 50, 50, 120};
  CHECK(offsets_ok(good, 3));
  CHECK(count_segments(good, 3, 16) == 4 + 0 + 5);
  CHECK(count_segments(good, 3, 1) == 120);
  const int64_t bad_start[] = {1, 50};
  CHECK(!offsets_ok(bad_start, 1));
  const int64_t decreasing[] = {0, 50, 40};
  CHECK(!offsets_ok(decreasing, 2));
  CHECK(!offsets_ok(nullptr, 1));
  CHECK(!offsets_ok(good, -1));
  const int64_t empty[] = {0};
  CHECK(offsets_ok(empty, 0) && count_segments(empty, 0, 8) == 0);
}

static void kd_ordering() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<float> u(-1000.0f, 1000.0f);
  for (int64_t n : {0, 1, 63, 64, 65, 127, 128, 1000, 4097, 20000}) {
    std::vector<float> keys(4 * (size_t)n);
    for (auto &k : keys) k = u(rng);
    if (n > 10) keys[4 * 3] = keys[4 * 5];  // a tie on the first axis
    std::vector<int32_t> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
    kd_order(idx.data(), n, keys.data(), 64);
    std::vector<char> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
      CHECK(idx[i] >= 0 && idx[i] < n && !seen[idx[i]]);
      seen[idx[i]] = 1;
    }
    // deterministic
    std::vector<int32_t> again(n);
    for (int64_t i = 0; i < n; ++i) again[i] = (int32_t)i;
    kd_order(again.data(), n, keys.data(), 64);
    CHECK(again == idx);
    // every split: its first m entries below the rest by (key on the range's
    // widest axis, index); later splits only reorder within the two parts
    std::vector<KdSplit> sp((size_t)kd_splits(n, 64, nullptr, nullptr, nullptr));
    kd_splits(n, 64, sp.data(), nullptr, nullptr);
    for (const KdSplit &s : sp) {
      float lo[4], hi[4];
      for (int f = 0; f < 4; ++f) {
        lo[f] = 1e30f;
        hi[f] = -1e30f;
      }
      for (int i = s.start; i < s.start + s.n; ++i)
        for (int f = 0; f < 4; ++f) {
          lo[f] = std::min(lo[f], keys[4 * (size_t)idx[i] + f]);
          hi[f] = std::max(hi[f], keys[4 * (size_t)idx[i] + f]);
        }
      int ax = 0;
      for (int f = 1; f < 4; ++f)
        if (hi[f] - lo[f] > hi[ax] - lo[ax]) ax = f;
      auto key = [&](int32_t a) { return std::make_pair(keys[4 * (size_t)a + ax], a); };
      std::pair<float, int32_t> lmax(-1e30f, -1), rmin(1e30f, 1 << 30);
      for (int i = s.start; i < s.start + s.m; ++i) lmax = std::max(lmax, key(idx[i]));
      for (int i = s.start + s.m; i < s.start + s.n; ++i) rmin = std::min(rmin, key(idx[i]));
      CHECK(lmax < rmin);
    }
    // inside every block the first half of each halving range below the
    // rest (checked on the top halving: the block's first n / 2 entries)
    for (int64_t b0 = 0; b0 < n; b0 += 64) {
      const int64_t c = std::min<int64_t>(64, n - b0);
      if (c < 2) continue;
      float lo[4], hi[4];
      for (int f = 0; f < 4; ++f) {
        lo[f] = 1e30f;
        hi[f] = -1e30f;
      }
      for (int64_t i = b0; i < b0 + c; ++i)
        for (int f = 0; f < 4; ++f) {
          lo[f] = std::min(lo[f], keys[4 * (size_t)idx[i] + f]);
          hi[f] = std::max(hi[f], keys[4 * (size_t)idx[i] + f]);
        }
      int ax = 0;
      for (int f = 1; f < 4; ++f)
        if (hi[f] - lo[f] > hi[ax] - lo[ax]) ax = f;
      auto key = [&](int32_t a) { return std::make_pair(keys[4 * (size_t)a + ax], a); };
      std::pair<float, int32_t> lmax(-1e30f, -1), rmin(1e30f, 1 << 30);
      for (int64_t i = b0; i < b0 + c / 2; ++i) lmax = std::max(lmax, key(idx[i]));
      for (int64_t i = b0 + c / 2; i < b0 + c; ++i) rmin = std::min(rmin, key(idx[i]));
      CHECK(lmax < rmin);
    }
  }
}

// The split list: level by level, disjoint ranges in order, every split
// longer than a block with m a positive multiple of the block below n; the
// ranges left unsplit at the end are at most a block long and all but the
// last are full.
static void kd_split_lists() {
  for (int64_t S : {0, 1, 64, 65, 128, 129, 200, 4097, 100000, 1234567}) {
    const int64_t ns = kd_splits(S, 64, nullptr, nullptr, nullptr);
    std::vector<KdSplit> sp((size_t)ns);
    int64_t lb[kKdMaxLevels + 1];
    int levels = -1;
    CHECK(kd_splits(S, 64, sp.data(), lb, &levels) == ns);
    CHECK(levels >= 0 && levels <= kKdMaxLevels && lb[levels] == ns);
    CHECK((S <= 64) == (ns == 0));
    // final ranges: replay the splits level by level
    std::vector<std::pair<int64_t, int64_t>> cur;
    if (S > 0) cur.push_back({0, S});
    for (int L = 0; L < levels; ++L) {
      int64_t end = 0;
      std::vector<std::pair<int64_t, int64_t>> next;
      size_t j = 0;
      for (int64_t i = lb[L]; i < lb[L + 1]; ++i) {
        const KdSplit &s = sp[(size_t)i];
        CHECK(s.start >= end && s.n > 64 && s.m > 0 && s.m < s.n && s.m % 64 == 0);
        end = s.start + s.n;
        CHECK(end <= S);
        while (j < cur.size() && cur[j].first < s.start) next.push_back(cur[j++]);
        CHECK(j < cur.size() && cur[j].first == s.start && cur[j].second == s.n);
        ++j;
        next.push_back({s.start, s.m});
        next.push_back({s.start + s.m, s.n - s.m});
      }
      while (j < cur.size()) next.push_back(cur[j++]);
      cur.swap(next);
    }
    int64_t pos = 0;
    for (size_t i = 0; i < cur.size(); ++i) {
      CHECK(cur[i].first == pos && cur[i].second <= 64);
      CHECK(i + 1 == cur.size() || cur[i].second == 64);
      pos += cur[i].second;
    }
    CHECK(pos == S);
  }
}

static void cache_lines() {
  char key[256];
  CHECK(cache_key(key, sizeof(key), "gfx950:sramecc+:xnack-", 64, 873000, 7400000) > 0);
  CHECK(std::strcmp(key, "batch gfx950_sramecc+_xnack- 64 873000 7400000") == 0);
  char tiny[8];
  CHECK(cache_key(tiny, sizeof(tiny), "gfx950", 1, 2, 3) == 0 && tiny[0] == '\0');
  std::string longarch(500, 'a');
  CHECK(cache_key(key, sizeof(key), longarch.c_str(), 1, 2, 3) == 0);
  CHECK(cache_key(key, sizeof(key), nullptr, 1, 2, 3) == 0);
  int cfg[3] = {0, 0, 0};
  CHECK(cache_key(key, sizeof(key), "gfx950", 4, 10, 20) > 0);
  std::string ok = std::string(key) + " 16 4 8\n";
  CHECK(cache_parse_line(ok.c_str(), key, cfg) && cfg[0] == 16 && cfg[1] == 4 && cfg[2] == 8);
  const char *bad_tails[] = {" 16 4", " 16 3 8", " 0 4 8", " 65 4 8", " 16 4 17", " x y z",
                             " 16 4 8 9", "", " 99999999999999999999 4 8", " -1 4 8"};
  for (const char *t : bad_tails) {
    std::string line = std::string(key) + t;
    CHECK(!cache_parse_line(line.c_str(), key, cfg));
  }
  std::string other = std::string(key) + "0 16 4 8";  // a longer key with the same prefix
  CHECK(!cache_parse_line(other.c_str(), key, cfg));
  CHECK(!cache_parse_line(nullptr, key, cfg) && !cache_parse_line("x", nullptr, cfg));
}

static void checkpoints() {
  const CkptDims dims{64, 6, 32, 128, 512, 4609};
  std::vector<unsigned char> payload(1000);
  for (size_t i = 0; i < payload.size(); ++i) payload[i] = (unsigned char)(i * 37 + 11);
  std::vector<unsigned char> buf(kCkptHeaderBytes + payload.size());
  ckpt_write_header(buf.data(), payload.size(), dims, fnv1a64(payload.data(), payload.size()));
  std::memcpy(buf.data() + kCkptHeaderBytes, payload.data(), payload.size());
  CHECK(ckpt_check(buf.data(), buf.size(), payload.size(), dims) == 0);
  // truncated and over-long buffers
  CHECK(ckpt_check(buf.data(), 10, payload.size(), dims) == -1);
  CHECK(ckpt_check(buf.data(), buf.size() - 1, payload.size(), dims) == -1);
  CHECK(ckpt_check(buf.data(), buf.size(), payload.size() + 1, dims) == -1);
  CHECK(ckpt_check(nullptr, buf.size(), payload.size(), dims) == -1);
  // every header byte and a payload byte matter
  for (size_t i = 0; i < kCkptHeaderBytes + 8; ++i) {
    std::vector<unsigned char> c = buf;
    c[i] ^= 0x40;
    const int r = ckpt_check(c.data(), c.size(), payload.size(), dims);
    if (i >= 56 && i < kCkptHeaderBytes) {
      CHECK(r == 0);  // reserved bytes
    } else {
      CHECK(r != 0);
    }
  }
  CkptDims other = dims;
  other.hidden = 32;
  CHECK(ckpt_check(buf.data(), buf.size(), payload.size(), other) == -4);
  // FNV-1a 64 of "a" (published test vector)
  CHECK(fnv1a64("a", 1) == 0xaf63dc4c8601ec8cull);
  CHECK(fnv1a64("", 0) == 0xcbf29ce484222325ull);
}

static void layouts() {
  for (int64_t n : {0, 1, 1000, 1000000}) {
    for (int64_t S : {n / 32, n / 32 + 1}) {
      const BuildLayout L = build_layout(n, S, 64, 64);
      const int64_t nb = (S + 63) / 64, ns = (nb + 63) / 64;
      // (offset, size) of every region, in layout order
      std::vector<std::pair<size_t, size_t>> r = {{L.pt4, 16 * n}, {L.pid, 4 * n}};
      for (int i = 0; i < 11; ++i) r.push_back({L.f[i], 4 * S});
      for (size_t o : {L.pstart, L.pcount, L.sorig, L.sfirst}) r.push_back({o, 4 * (size_t)S});
      r.push_back({L.box, 32 * (size_t)nb});
      r.push_back({L.sbox, 32 * (size_t)ns});
      for (int i = 0; i < 11; ++i) r.push_back({L.tf[i], 4 * S});
      r.push_back({L.tstart, 4 * S});
      r.push_back({L.tcf, 4 * S});
      r.push_back({L.keys, 16 * S});
      r.push_back({L.perm, 4 * S});
      r.push_back({L.dpstart, 4 * S});
      r.push_back({L.kdsplits, sizeof(KdSplit) * (size_t)kd_splits(S, 64, nullptr, nullptr, nullptr)});
      r.push_back({L.status, 32});
      for (size_t i = 0; i < r.size(); ++i) {
        CHECK(r[i].first % 256 == 0);
        if (i + 1 < r.size()) CHECK(r[i].first + r[i].second <= r[i + 1].first);
      }
      CHECK(r.back().first + r.back().second <= L.total && L.total % 256 == 0);
    }
  }
}

int main() {
  layouts();
  offsets_and_counts();
  kd_ordering();
  kd_split_lists();
  cache_lines();
  checkpoints();
  std::printf("host ok\n");
  return 0;
}
