// shake.cpp -- SHAKE-256 (FIPS 202) and the seeded samplers of key generation
// and encryption.  A stream is SHAKE-256 over le64(seed) || le32(domain) ||
// le64(index), read as little-endian 64-bit words.
#include <cstring>

#include "bm_internal.hpp"

namespace bm {
namespace {

constexpr u64 kRC[24] = {
    0x0000000000000001ULL, 0x0000000000008082ULL, 0x800000000000808aULL, 0x8000000080008000ULL,
    0x000000000000808bULL, 0x0000000080000001ULL, 0x8000000080008081ULL, 0x8000000000008009ULL,
    0x000000000000008aULL, 0x0000000000000088ULL, 0x0000000080008009ULL, 0x000000008000000aULL,
    0x000000008000808bULL, 0x800000000000008bULL, 0x8000000000008089ULL, 0x8000000000008003ULL,
    0x8000000000008002ULL, 0x8000000000000080ULL, 0x000000000000800aULL, 0x800000008000000aULL,
    0x8000000080008081ULL, 0x8000000000008080ULL, 0x0000000080000001ULL, 0x8000000080008008ULL};
// rotation offset and pi destination, lane index x + 5y
constexpr int kRho[25] = {0, 1, 62, 28, 27, 36, 44, 6, 55, 20, 3, 10, 43,
                          25, 39, 41, 45, 15, 21, 8, 18, 2, 61, 56, 14};

inline u64 rol(u64 v, int r) { return r == 0 ? v : (v << r) | (v >> (64 - r)); }

void permute(u64 s[25]) {
  for (int round = 0; round < 24; ++round) {
    u64 C[5];
    for (int x = 0; x < 5; ++x) C[x] = s[x] ^ s[x + 5] ^ s[x + 10] ^ s[x + 15] ^ s[x + 20];
    for (int x = 0; x < 5; ++x) {
      u64 D = C[(x + 4) % 5] ^ rol(C[(x + 1) % 5], 1);
      for (int y = 0; y < 25; y += 5) s[x + y] ^= D;
    }
    u64 B[25];
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) {
        int src = x + 5 * y;
        int dx = y, dy = (2 * x + 3 * y) % 5;
        B[dx + 5 * dy] = rol(s[src], kRho[src]);
      }
    for (int y = 0; y < 25; y += 5)
      for (int x = 0; x < 5; ++x) s[x + y] = B[x + y] ^ (~B[(x + 1) % 5 + y] & B[(x + 2) % 5 + y]);
    s[0] ^= kRC[round];
  }
}

class Shake {
 public:
  static constexpr size_t kRate = 136;
  void absorb_final(const uint8_t* in, size_t len) {
    std::memset(s_, 0, sizeof(s_));
    while (len >= kRate) {
      xor_block(in, kRate);
      permute(s_);
      in += kRate;
      len -= kRate;
    }
    uint8_t blk[kRate] = {0};
    std::memcpy(blk, in, len);
    blk[len] ^= 0x1F;
    blk[kRate - 1] ^= 0x80;
    xor_block(blk, kRate);
    permute(s_);
    pos_ = 0;
  }
  void squeeze(uint8_t* out, size_t len) {
    while (len) {
      if (pos_ == kRate) {
        permute(s_);
        pos_ = 0;
      }
      size_t take = std::min(len, kRate - pos_);
      for (size_t i = 0; i < take; ++i) out[i] = (uint8_t)(s_[(pos_ + i) >> 3] >> (8 * ((pos_ + i) & 7)));
      pos_ += take;
      out += take;
      len -= take;
    }
  }
  u64 word() {
    // words are 8-byte aligned inside the rate (136 = 17 * 8)
    if (pos_ == kRate) {
      permute(s_);
      pos_ = 0;
    }
    u64 w = s_[pos_ >> 3];
    pos_ += 8;
    return w;
  }

 private:
  void xor_block(const uint8_t* p, size_t len) {
    for (size_t i = 0; i < len; ++i) s_[i >> 3] ^= (u64)p[i] << (8 * (i & 7));
  }
  u64 s_[25];
  size_t pos_ = 0;
};

void open_stream(Shake& sh, u64 seed, u32 domain, u64 index) {
  uint8_t msg[20];
  for (int i = 0; i < 8; ++i) msg[i] = (uint8_t)(seed >> (8 * i));
  for (int i = 0; i < 4; ++i) msg[8 + i] = (uint8_t)(domain >> (8 * i));
  for (int i = 0; i < 8; ++i) msg[12 + i] = (uint8_t)(index >> (8 * i));
  sh.absorb_final(msg, sizeof(msg));
}

}  // namespace

void shake256(const uint8_t* in, size_t inlen, uint8_t* out, size_t outlen) {
  Shake sh;
  sh.absorb_final(in, inlen);
  sh.squeeze(out, outlen);
}

void sample_ternary(u64 seed, u32 domain, u64 index, size_t n, int64_t* out) {
  Shake sh;
  open_stream(sh, seed, domain, index);
  const u64 limit = 0xFFFFFFFFFFFFFFFFULL;   // 3 * floor(2^64 / 3)
  for (size_t i = 0; i < n;) {
    u64 u = sh.word();
    if (u >= limit) continue;
    out[i++] = (int64_t)(u % 3) - 1;
  }
}

void sample_gauss(const Ctx& c, u64 seed, u32 domain, u64 index, size_t n, int64_t* out) {
  Shake sh;
  open_stream(sh, seed, domain, index);
  const int half = (int)c.cdt.size() / 2;
  for (size_t i = 0; i < n; ++i) {
    u64 u = sh.word();
    // binary search: number of table entries <= u
    size_t lo = 0, hi = c.cdt.size();
    while (lo < hi) {
      size_t mid = (lo + hi) / 2;
      if (c.cdt[mid] <= u) lo = mid + 1;
      else hi = mid;
    }
    out[i] = (int64_t)lo - half;
  }
}

void sample_uniform(u64 seed, u32 domain, u64 index, const u64* qs, size_t nq, size_t n, u64* out) {
  Shake sh;
  open_stream(sh, seed, domain, index);
  for (size_t l = 0; l < nq; ++l) {
    const u64 q = qs[l];
    const int bits = 64 - __builtin_clzll(q);
    const u64 mask = bits == 64 ? ~0ULL : ((1ULL << bits) - 1);
    u64* row = out + l * n;
    for (size_t i = 0; i < n;) {
      u64 u = sh.word() & mask;
      if (u < q) row[i++] = u;
    }
  }
}

}  // namespace bm
