// Host-only logic of the library (declared in host.h): no HIP here.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

namespace tnn {
namespace host {

bool offsets_ok(const int64_t *off, int64_t n_traj) {
  if (!off || n_traj < 0 || off[0] != 0) return false;
  for (int64_t j = 0; j < n_traj; ++j)
    if (off[j + 1] < off[j]) return false;
  return true;
}

int64_t count_segments(const int64_t *off, int64_t n_traj, int32_t K) {
  int64_t s = 0;
  for (int64_t j = 0; j < n_traj; ++j) s += (off[j + 1] - off[j] + K - 1) / K;
  return s;
}

BuildLayout build_layout(int64_t n, int64_t S, int64_t block, int64_t superblock) {
  BuildLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  const int64_t nb = (S + block - 1) / block;
  L.pt4 = take(16 * (size_t)n);
  L.pid = take(4 * (size_t)n);
  for (int i = 0; i < 11; ++i) L.f[i] = take(4 * (size_t)S);
  L.pstart = take(4 * (size_t)S);
  L.pcount = take(4 * (size_t)S);
  L.sorig = take(4 * (size_t)S);
  L.sfirst = take(4 * (size_t)S);
  L.box = take(4 * 8 * (size_t)nb);
  L.sbox = take(4 * 8 * (size_t)((nb + superblock - 1) / superblock));
  for (int i = 0; i < 11; ++i) L.tf[i] = take(4 * (size_t)S);
  L.tstart = take(4 * (size_t)S);
  L.tcf = take(4 * (size_t)S);
  L.keys = take(16 * (size_t)S);
  L.perm = take(4 * (size_t)S);
  L.dpstart = take(4 * (size_t)S);
  L.kdsplits = take(sizeof(KdSplit) * (size_t)kd_splits(S, block, nullptr, nullptr, nullptr));
  L.status = take(32);
  L.total = o;
  return L;
}

int64_t kd_splits(int64_t S, int64_t block, KdSplit *splits, int64_t *level_begin,
                  int *n_levels) {
  // ranges of the current level: (start, n), in order
  std::vector<std::pair<int64_t, int64_t>> cur, next;
  if (S > 0) cur.push_back({0, S});
  int64_t count = 0;
  int levels = 0;
  for (;;) {
    next.clear();
    const int64_t first = count;
    for (const auto &r : cur) {
      const int64_t n = r.second;
      if (n <= block) {
        next.push_back(r);
        continue;
      }
      int64_t m = ((n / 2 + block - 1) / block) * block;
      if (m >= n) m = (n - 1) / block * block;
      if (splits) splits[count] = KdSplit{(int32_t)r.first, (int32_t)n, (int32_t)m, 0};
      ++count;
      next.push_back({r.first, m});
      next.push_back({r.first + m, n - m});
    }
    if (count == first) break;
    if (level_begin) level_begin[levels] = first;
    ++levels;
    cur.swap(next);
  }
  if (level_begin) level_begin[levels] = count;
  if (n_levels) *n_levels = levels;
  return count;
}

void kd_order(int32_t *idx, int64_t n, const float *keys, int64_t block) {
  std::vector<int32_t> tmp;
  // r[0, len) into its m smallest by (key on the widest axis, index) and
  // the rest, each part keeping its order
  auto split_range = [&](int32_t *r, int64_t len, int64_t m) {
    float lo[4], hi[4];
    for (int f = 0; f < 4; ++f) {
      lo[f] = INFINITY;
      hi[f] = -INFINITY;
    }
    for (int64_t i = 0; i < len; ++i)
      for (int f = 0; f < 4; ++f) {
        const float v = keys[4 * (size_t)r[i] + f];
        lo[f] = std::min(lo[f], v);
        hi[f] = std::max(hi[f], v);
      }
    int axis = 0;
    for (int f = 1; f < 4; ++f)
      if (hi[f] - lo[f] > hi[axis] - lo[axis]) axis = f;
    auto less = [&](int32_t a, int32_t b) {
      const float ka = keys[4 * (size_t)a + axis], kb = keys[4 * (size_t)b + axis];
      return ka < kb || (ka == kb && a < b);
    };
    tmp.assign(r, r + len);
    std::nth_element(tmp.begin(), tmp.begin() + m, tmp.end(), less);
    const int32_t pivot = tmp[(size_t)m];
    std::stable_partition(r, r + len, [&](int32_t a) { return less(a, pivot); });
  };
  const int64_t ns = kd_splits(n, block, nullptr, nullptr, nullptr);
  std::vector<KdSplit> sp((size_t)ns);
  kd_splits(n, block, sp.data(), nullptr, nullptr);
  for (const KdSplit &s : sp) split_range(idx + s.start, s.n, s.m);
  // inside each block (the last one shorter) the splits go on down to single
  // entries, m = n / 2, level by level
  for (int64_t b0 = 0; b0 < n; b0 += block) {
    const int64_t c = std::min<int64_t>(block, n - b0);
    std::vector<std::pair<int64_t, int64_t>> cur{{b0, c}}, next;
    bool any = true;
    while (any) {
      any = false;
      next.clear();
      for (const auto &rg : cur) {
        if (rg.second < 2) {
          next.push_back(rg);
          continue;
        }
        any = true;
        split_range(idx + rg.first, rg.second, rg.second / 2);
        next.push_back({rg.first, rg.second / 2});
        next.push_back({rg.first + rg.second / 2, rg.second - rg.second / 2});
      }
      cur.swap(next);
    }
  }
}

size_t cache_key(char *out, size_t cap, const char *arch, int n_items, long long total_q,
                 long long total_p) {
  if (!out || cap == 0) return 0;
  out[0] = '\0';
  if (!arch) return 0;
  // the architecture name may carry ':'-separated feature suffixes: keep the
  // key one token per field
  char a[128];
  size_t n = 0;
  for (; arch[n] && n + 1 < sizeof(a); ++n) {
    const char c = arch[n];
    a[n] = (c == ':' || c == ' ' || c == '\t' || c == '\n' || c == '\r') ? '_' : c;
  }
  if (arch[n]) return 0;  // longer than any architecture name
  a[n] = '\0';
  const int len = std::snprintf(out, cap, "batch %s %d %lld %lld", a, n_items, total_q, total_p);
  if (len < 0 || (size_t)len >= cap) {
    out[0] = '\0';
    return 0;
  }
  return (size_t)len;
}

static bool parse_int(const char *&p, long lo, long hi, int &out) {
  while (*p == ' ' || *p == '\t') ++p;
  char *end = nullptr;
  const long v = std::strtol(p, &end, 10);
  if (end == p || v < lo || v > hi) return false;
  p = end;
  out = (int)v;
  return true;
}

bool cache_parse_line(const char *line, const char *key, int cfg[3]) {
  if (!line || !key || !cfg) return false;
  const size_t kl = std::strlen(key);
  if (kl == 0 || std::strncmp(line, key, kl) != 0 || line[kl] != ' ') return false;
  const char *p = line + kl;
  int c = 0, w = 0, b = 0;
  if (!parse_int(p, 1, 64, c) || !parse_int(p, 1, 8, w) || !parse_int(p, 1, 16, b)) return false;
  if (!(w == 1 || w == 2 || w == 4 || w == 8)) return false;
  while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') ++p;
  if (*p != '\0') return false;
  cfg[0] = c;
  cfg[1] = w;
  cfg[2] = b;
  return true;
}

uint64_t fnv1a64(const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  uint64_t h = 0xcbf29ce484222325ull;  // FNV-1a 64-bit offset basis and prime
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

static const char kMagic[8] = {'T', 'N', 'N', 'R', 'A', 'D', 'M', '\0'};

void ckpt_write_header(void *dst, uint64_t payload_bytes, const CkptDims &dims, uint64_t checksum) {
  unsigned char h[kCkptHeaderBytes];
  std::memset(h, 0, sizeof(h));
  std::memcpy(h, kMagic, 8);
  const uint32_t version = kCkptVersion, hb = (uint32_t)kCkptHeaderBytes;
  std::memcpy(h + 8, &version, 4);
  std::memcpy(h + 12, &hb, 4);
  std::memcpy(h + 16, &payload_bytes, 8);
  const uint32_t d[6] = {dims.hidden, dims.inputs, dims.grid, dims.start_xy, dims.start_t,
                         dims.nparams};
  std::memcpy(h + 24, d, 24);
  std::memcpy(h + 48, &checksum, 8);
  std::memcpy(dst, h, sizeof(h));
}

int ckpt_check(const void *buf, size_t bytes, uint64_t payload_bytes, const CkptDims &dims) {
  if (!buf || bytes < kCkptHeaderBytes) return -1;
  const unsigned char *h = static_cast<const unsigned char *>(buf);
  if (std::memcmp(h, kMagic, 8) != 0) return -2;
  uint32_t version = 0, hb = 0;
  std::memcpy(&version, h + 8, 4);
  std::memcpy(&hb, h + 12, 4);
  if (version != kCkptVersion || hb != kCkptHeaderBytes) return -3;
  uint64_t pb = 0;
  std::memcpy(&pb, h + 16, 8);
  if (pb != payload_bytes || bytes != kCkptHeaderBytes + payload_bytes) return -1;
  uint32_t d[6];
  std::memcpy(d, h + 24, 24);
  if (d[0] != dims.hidden || d[1] != dims.inputs || d[2] != dims.grid || d[3] != dims.start_xy ||
      d[4] != dims.start_t || d[5] != dims.nparams)
    return -4;
  uint64_t sum = 0;
  std::memcpy(&sum, h + 48, 8);
  if (fnv1a64(h + kCkptHeaderBytes, payload_bytes) != sum) return -5;
  return 0;
}

}  // namespace host
}  // namespace tnn
