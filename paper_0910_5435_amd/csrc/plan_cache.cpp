// Plan cache: the butterflies of a plan on disk, one checksummed record per (order, parity),
// so that a later sht_plan_ex with the same (l, eps, leaf width) skips the precompute of
// Section 4 (the paper's t_comp, which grows like n^2) and an interrupted build resumes at
// the first pair it had not finished.
//
// File <cache_dir>/sht_plan_l<l>_C<C>_e<eps bits>_v<format>.cache:
//   header  "SHTPLAN\0", format, l, C, number of pairs, eps (FP64 bits), CRC-32 of the above;
//   records in increasing pair index mp = 2m + p, each: mp (u32), payload bytes (u64),
//   payload (BfTree::save), CRC-32 of (mp, size, payload).
// A record whose checksum, pair index or payload does not match ends the valid prefix; the
// builder cuts the file there and rebuilds from that pair on.  Records are appended as each
// batch of pairs is built, so a crash loses at most the batch in progress.
#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "interp_decomp.h"
#include "plan_cache.h"
#include "sht.h"

namespace sht {

namespace {

constexpr char kMagic[8] = {'S', 'H', 'T', 'P', 'L', 'A', 'N', '\0'};
constexpr uint32_t kFormat = 1;
constexpr size_t kHeaderBytes = 8 + 4 + 4 + 4 + 4 + 8 + 4;

// CRC-32 with the reflected polynomial 0xEDB88320 (the checksum of zip/PNG/Ethernet),
// computed bytewise from a 256-entry table.
struct CrcTable {
  uint32_t t[256];
  CrcTable() {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      t[i] = c;
    }
  }
};
const CrcTable& crc_table() {
  static const CrcTable tab;
  return tab;
}

uint32_t crc_update(uint32_t crc, const void* data, size_t n) {
  const CrcTable& tab = crc_table();
  const unsigned char* p = static_cast<const unsigned char*>(data);
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) crc = tab.t[(crc ^ p[i]) & 0xFFu] ^ (crc >> 8);
  return ~crc;
}

std::vector<unsigned char> header_bytes(int l, int C, int npairs, double eps) {
  std::vector<unsigned char> h(kHeaderBytes);
  unsigned char* p = h.data();
  std::memcpy(p, kMagic, 8);
  const uint32_t fmt = kFormat;
  const int32_t v[3] = {l, C, npairs};
  std::memcpy(p + 8, &fmt, 4);
  std::memcpy(p + 12, v, 12);
  std::memcpy(p + 24, &eps, 8);
  const uint32_t crc = crc_update(0, p, 32);
  std::memcpy(p + 32, &crc, 4);
  return h;
}

}  // namespace

uint32_t cache_crc32(const void* data, size_t n) { return crc_update(0, data, n); }

PairShape pair_shape(int l, int C, int mp) {
  const int m = mp / 2, n = 2 * l - m;
  const int n0 = (n + 1) / 2, n1 = n / 2;
  return {l, mp % 2 ? n1 : n0, butterfly_depth(n0, C)};
}

std::string cache_path(const char* dir, int l, double eps, int C) {
  uint64_t bits = 0;
  std::memcpy(&bits, &eps, 8);
  char name[160];
  std::snprintf(name, sizeof(name), "/sht_plan_l%d_C%d_e%016llx_v%u.cache", l, C,
                static_cast<unsigned long long>(bits), kFormat);
  return std::string(dir) + name;
}

int cache_scan(const char* dir, int l, double eps, int C, int npairs,
               const std::vector<PairShape>* shapes, std::vector<BfTree>* trees, CacheScan& out) {
  out = CacheScan{};
  if (!dir || l < 1 || C < 1 || npairs < 0) return SHT_EINVAL;
  const std::string path = cache_path(dir, l, eps, C);
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return SHT_EINVAL;
  out.exists = true;
  std::vector<unsigned char> h(kHeaderBytes);
  const std::vector<unsigned char> want = header_bytes(l, C, npairs, eps);
  if (std::fread(h.data(), 1, kHeaderBytes, f) != kHeaderBytes || h != want) {
    std::fclose(f);
    out.corrupt = true;
    return SHT_ECORRUPT;
  }
  out.valid_bytes = static_cast<long long>(kHeaderBytes);
  std::vector<unsigned char> payload;
  int rc = SHT_OK;
  for (int mp = 0; mp < npairs; ++mp) {
    uint32_t rmp = 0, crc = 0;
    uint64_t size = 0;
    if (std::fread(&rmp, 4, 1, f) != 1) break;  // clean end: the valid prefix is complete
    if (std::fread(&size, 8, 1, f) != 1 || rmp != static_cast<uint32_t>(mp) || size > (uint64_t(1) << 34)) {
      rc = SHT_ECORRUPT;
      break;
    }
    payload.resize(size);
    if ((size && std::fread(payload.data(), 1, size, f) != size) || std::fread(&crc, 4, 1, f) != 1) {
      rc = SHT_ECORRUPT;
      break;
    }
    uint32_t c = crc_update(0, &rmp, 4);
    c = crc_update(c, &size, 8);
    c = crc_update(c, payload.data(), size);
    if (c != crc) {
      rc = SHT_ECORRUPT;
      break;
    }
    if (shapes && trees) {
      const PairShape& s = (*shapes)[mp];
      if (!(*trees)[mp].load(payload.data(), size, s.rows, s.cols, C, s.L, eps)) {
        rc = SHT_ECORRUPT;
        break;
      }
    }
    out.valid_pairs = mp + 1;
    out.valid_bytes += static_cast<long long>(4 + 8 + size + 4);
  }
  // anything after the last expected record is also foreign
  if (rc == SHT_OK && out.valid_pairs == npairs && std::fgetc(f) != EOF) rc = SHT_ECORRUPT;
  std::fclose(f);
  out.corrupt = rc == SHT_ECORRUPT;
  return rc;
}

CacheWriter::~CacheWriter() {
  if (f_) std::fclose(static_cast<FILE*>(f_));
}

int CacheWriter::open(const char* dir, int l, double eps, int C, int npairs, long long keep_bytes) {
  const std::string path = cache_path(dir, l, eps, C);
  if (keep_bytes < static_cast<long long>(kHeaderBytes)) {
    FILE* f = std::fopen(path.c_str(), "wb");
    if (!f) return SHT_EINVAL;
    const std::vector<unsigned char> h = header_bytes(l, C, npairs, eps);
    if (std::fwrite(h.data(), 1, h.size(), f) != h.size()) {
      std::fclose(f);
      return SHT_EINVAL;
    }
    f_ = f;
    return std::fflush(f) == 0 ? SHT_OK : SHT_EINVAL;
  }
  // keep the valid prefix, drop whatever follows it (a corrupt or foreign tail)
  if (truncate(path.c_str(), static_cast<off_t>(keep_bytes)) != 0) return SHT_EINVAL;
  FILE* f = std::fopen(path.c_str(), "ab");
  if (!f) return SHT_EINVAL;
  f_ = f;
  return SHT_OK;
}

int CacheWriter::append(int mp, const BfTree& tree) {
  FILE* f = static_cast<FILE*>(f_);
  if (!f) return SHT_EINVAL;
  buf_.clear();
  tree.save(buf_);
  const uint32_t rmp = static_cast<uint32_t>(mp);
  const uint64_t size = buf_.size();
  uint32_t c = crc_update(0, &rmp, 4);
  c = crc_update(c, &size, 8);
  c = crc_update(c, buf_.data(), buf_.size());
  if (std::fwrite(&rmp, 4, 1, f) != 1 || std::fwrite(&size, 8, 1, f) != 1 ||
      (size && std::fwrite(buf_.data(), 1, size, f) != size) || std::fwrite(&c, 4, 1, f) != 1)
    return SHT_EINVAL;
  return SHT_OK;
}

int CacheWriter::flush() {
  FILE* f = static_cast<FILE*>(f_);
  return f && std::fflush(f) == 0 ? SHT_OK : SHT_EINVAL;
}

}  // namespace sht
