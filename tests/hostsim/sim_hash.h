// Hashes shared by the host-side fake device and the scheduler test driver.
#pragma once
#include <cstdint>
#include <cstring>

namespace sim {

inline uint64_t splitmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Identity of a table: its parameters as the build job carries them.
inline uint64_t table_tag(const double q[4], int k, int mode) {
  uint64_t h = 0x1234;
  for (int i = 0; i < 4; ++i) {
    uint64_t v;
    std::memcpy(&v, &q[i], 8);
    h = splitmix(h ^ v);
  }
  return splitmix(h ^ (static_cast<uint64_t>(static_cast<uint32_t>(k)) << 8) ^ static_cast<uint64_t>(mode));
}

// What the fake generation XORs into a request's digest for edge e.
inline uint64_t edge_word(uint64_t e, uint64_t seed, uint64_t tag) { return splitmix(e ^ splitmix(seed ^ tag)); }

// Build results the fake device reports as failed: a = 0.125 exactly.
inline bool build_fails(const double q[4]) { return q[0] == 0.125; }

}  // namespace sim
