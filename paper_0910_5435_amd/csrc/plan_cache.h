// Plan cache (plan_cache.cpp): checksummed per-pair butterfly records on disk.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "interp_decomp.h"

namespace sht {

// Shape of the butterfly of one (order, parity) pair: Q^{(m,p)} is rows x cols, depth L.
struct PairShape {
  int rows, cols, L;
};

struct CacheScan {
  bool exists = false;      // the file was found
  bool corrupt = false;     // a header or record failed its check (the valid prefix ends there)
  int valid_pairs = 0;      // records 0 .. valid_pairs - 1 are intact
  long long valid_bytes = 0;  // bytes of the header plus those records
};

// Shape of pair mp = 2m + p of a plan of bandlimit l and leaf width C: l rows (positive nodes),
// the degrees m + p + 2j <= 2l - 1 as columns, depth L = ceil(log2(ceil(n_0 / C))) shared by
// both parities of an order (n_0: the parity-0 column count).
PairShape pair_shape(int l, int C, int mp);

std::string cache_path(const char* dir, int l, double eps, int C);
uint32_t cache_crc32(const void* data, size_t n);

// Reads the cache file of (l, eps, C) with npairs expected records.  With shapes and trees,
// record mp is loaded into (*trees)[mp] for every mp of the valid prefix.  Returns SHT_OK
// (the records present are intact, possibly fewer than npairs), SHT_ECORRUPT (out.valid_pairs
// counts the intact prefix) or SHT_EINVAL (no such file, bad arguments).
int cache_scan(const char* dir, int l, double eps, int C, int npairs, const std::vector<PairShape>* shapes,
               std::vector<BfTree>* trees, CacheScan& out);

// Appends records to the cache file, keeping its first keep_bytes (a valid prefix found by
// cache_scan; fewer than a header's bytes starts a new file).
class CacheWriter {
 public:
  CacheWriter() = default;
  CacheWriter(const CacheWriter&) = delete;
  CacheWriter& operator=(const CacheWriter&) = delete;
  ~CacheWriter();
  int open(const char* dir, int l, double eps, int C, int npairs, long long keep_bytes);
  int append(int mp, const BfTree& tree);
  int flush();
  bool is_open() const { return f_ != nullptr; }

 private:
  void* f_ = nullptr;  // FILE*
  std::vector<unsigned char> buf_;
};

}  // namespace sht
