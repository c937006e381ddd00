// Host-only logic of the library, free of HIP: validation of the trajectory
// offsets, the spatial ordering of segments into blocks, the autotuner's
// cache format and the radius-model checkpoint header.  Compiled into
// libtnn, and on its own with g++ under the address and undefined-behaviour
// sanitizers by the CPU tests.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace tnn {
namespace host {

// offsets[0] = 0 and non-decreasing over n_traj + 1 entries.
bool offsets_ok(const int64_t *off, int64_t n_traj);

// Segments produced by cutting every trajectory into runs of K points (the
// last run of a trajectory may be shorter).
int64_t count_segments(const int64_t *off, int64_t n_traj, int32_t K);

// Byte offsets, 256-byte aligned, of the arrays of an index of n points and
// S segments inside the caller's buffer: points in index order (float4 and
// caller id), the 11 float32 segment fields, first slot, member count,
// trajectory-order number and first-of-trajectory flag per segment, block
// and superblock boxes (8 float32 each), and the build's temporaries.
struct BuildLayout {
  size_t pt4, pid;
  size_t f[11], pstart, pcount, sorig, sfirst;
  size_t box, sbox;
  size_t tf[11], tstart, tcf, keys, perm, dpstart, kdsplits, status;
  size_t total;
};
BuildLayout build_layout(int64_t n, int64_t S, int64_t block, int64_t superblock);

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// The kd order of segments into blocks: a range of the order longer than
// `block` splits along the widest of its 4 key axes into its m smallest
// entries (by key, ties by index) and the rest, m = n / 2 rounded up to a
// multiple of `block` (so every block but the last is full), each part
// keeping the order the range had; the parts split again until no range is
// longer than `block`; each final range (a block, the last one shorter) is
// then sorted along its own widest axis (ties by index).  The splits depend
// on the entry count alone: level by level, split ranges only (a range of at
// most `block` entries stays as it is).  The device builds the order with
// these splits.
struct KdSplit {
  int32_t start, n, m, pad;
};
// Splits of the kd order of S entries, level after level; level L holds
// splits[level_begin[L] .. level_begin[L + 1]).  Returns the split count
// (splits and level_begin may be null to count only; level_begin then needs
// one more entry than there are levels, at most 64).
int64_t kd_splits(int64_t S, int64_t block, KdSplit *splits, int64_t *level_begin,
                  int *n_levels);
constexpr int kKdMaxLevels = 64;

// The same order on the host (reference for the tests): idx[0, n) is
// reordered in place; keys[4 * idx[i] + f].
void kd_order(int32_t *idx, int64_t n, const float *keys, int64_t block);

// Autotuner cache: one line per tuned problem, "<key> <chunk> <waves> <blocks>".
// The key names the device architecture (':' replaced by '_'), the item
// count, the total queries and the total points.  Returns the key length, or
// 0 when it does not fit in cap bytes (including the terminating zero).
size_t cache_key(char *out, size_t cap, const char *arch, int n_items, long long total_q,
                 long long total_p);
// True when `line` starts with `key` followed by a space and three integers
// in range (chunk 1..64, waves 1, 2, 4 or 8, blocks per CU 1..16).
bool cache_parse_line(const char *line, const char *key, int cfg[3]);

// Radius-model checkpoint: a 64-byte header followed by the model's device
// bytes.  Header (little endian): magic "TNNRADM\0", version, header size,
// payload size, the model's dimensions (hidden units, inputs, density grid,
// start grid x/y and t, parameter count), FNV-1a 64 of the payload.
constexpr uint32_t kCkptVersion = 1;
constexpr size_t kCkptHeaderBytes = 64;
struct CkptDims {
  uint32_t hidden, inputs, grid, start_xy, start_t, nparams;
};
uint64_t fnv1a64(const void *p, size_t n);
void ckpt_write_header(void *dst, uint64_t payload_bytes, const CkptDims &dims, uint64_t checksum);
// 0 when buf[0, bytes) is a complete checkpoint of this version with these
// dimensions and payload size and a matching checksum; a negative code naming
// the first problem otherwise (-1 size, -2 magic, -3 version, -4 dimensions,
// -5 checksum).
int ckpt_check(const void *buf, size_t bytes, uint64_t payload_bytes, const CkptDims &dims);

}  // namespace host
}  // namespace tnn
