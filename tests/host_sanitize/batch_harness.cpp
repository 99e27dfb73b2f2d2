// Host path of the vector batch (mont_batch_reserve / update / mul / destroy)
// under the address and undefined-behaviour sanitizers, with the HIP runtime
// replaced by the host stand-in next to this file: every staging write, every
// upload length and every buffer lifetime is checked, and the emulated kernel
// reads the uploaded descriptors and operands through the same pointers the
// GPU would.  Sequences: the uneven 4096-vector batch of the bench (the
// capacity exactly full), batches on both sides of the 16-vector inline
// limit, empty batches, repeated updates without a launch in between, and
// the error paths.
#include "../../paper_1609_00999_amd/csrc/batch.hip"

#include <stdio.h>

#include <random>
#include <vector>

namespace {

int failures = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    printf("FAIL %s\n", what);
    failures++;
  }
}

// -P^-1 mod 2^32 by Newton's iteration (x <- x (2 - P x) doubles the correct bits).
uint32_t neg_inverse(uint32_t P) {
  uint32_t x = P;
  for (int i = 0; i < 5; i++) x *= 2u - P * x;
  return 0u - x;
}

struct Vec {
  std::vector<uint32_t> a, b, out;   // storage; the vector starts at element off
  size_t off = 0, n = 0;
  uint32_t P = 0;
};

// out[j] R = a[j] b[j] (mod P) and out[j] < P: the defining property of a
// Montgomery product, checked with 64-bit remainders.
bool product_ok(const Vec& v) {
  for (size_t j = v.off; j < v.off + v.n; j++) {
    const uint64_t lhs = ((uint64_t)v.out[j] << 32) % v.P;
    const uint64_t rhs = (uint64_t)v.a[j] * v.b[j] % v.P;
    if (v.out[j] >= v.P || lhs != rhs) return false;
  }
  return true;
}

bool run_batch(mont_batch* b, std::vector<Vec>& vs, std::mt19937_64& rng, int count, uint64_t maxn,
               bool misalign) {
  static const uint32_t primes[] = {2013265921u, 1811939329u, 2113929217u, 998244353u, 17u};
  vs.assign(count, Vec());
  std::vector<mont_vec_desc> d(count > 0 ? count : 1);
  for (int i = 0; i < count; i++) {
    Vec& v = vs[i];
    v.P = primes[rng() % 5];
    v.n = (size_t)(rng() % (maxn + 1));
    v.off = misalign ? (size_t)(i & 3) : 0;      // start 4, 8 or 12 bytes into a 16-byte line
    v.a.resize(v.n + v.off);
    v.b.resize(v.n + v.off);
    v.out.assign(v.n + v.off, 0xFFFFFFFFu);
    for (size_t j = 0; j < v.n + v.off; j++) {
      v.a[j] = (uint32_t)(rng() % v.P);
      v.b[j] = (uint32_t)(rng() % v.P);
    }
    d[i].a = v.a.data() + v.off;
    d[i].b = v.b.data() + v.off;
    d[i].out = v.out.data() + v.off;
    d[i].n = v.n;
    d[i].P = v.P;
    d[i].Pprime = neg_inverse(v.P);
  }
  if (mont_batch_update(b, d.data(), count, nullptr) != MONT_OK) return false;
  if (mont_batch_mul(b, nullptr) != MONT_OK) return false;
  for (int i = 0; i < count; i++)
    if (!product_ok(vs[i])) return false;
  return true;
}

}  // namespace

int main() {
  std::mt19937_64 rng(20240611);
  std::vector<Vec> vs;
  // the bench's shape: capacity 4096, every slot used, uneven lengths
  mont_batch* b = nullptr;
  check(mont_batch_reserve(4096, &b) == MONT_OK, "reserve 4096");
  check(run_batch(b, vs, rng, 4096, 9000, false), "4096 uneven vectors, capacity full");
  check(run_batch(b, vs, rng, 3, 20000, false), "3 vectors (descriptors in the launch)");
  check(run_batch(b, vs, rng, 17, 5000, true), "17 vectors, misaligned (uploaded)");
  check(run_batch(b, vs, rng, 16, 5000, true), "16 vectors, misaligned (in the launch)");
  check(run_batch(b, vs, rng, 0, 10, false), "empty batch");
  check(run_batch(b, vs, rng, 4096, 3, false), "4096 tiny vectors");
  // updates without a launch in between reuse the staging block
  for (int rep = 0; rep < 20; rep++) {
    const int count = (int)(rng() % 4097);
    check(run_batch(b, vs, rng, count, 6000, rep & 1), "random batch");
  }
  mont_vec_desc bad = {nullptr, nullptr, nullptr, 5, 2013265921u, neg_inverse(2013265921u)};
  check(mont_batch_update(b, &bad, 1, nullptr) == MONT_EINVAL, "null operands with n > 0");
  std::vector<mont_vec_desc> many(4097, bad);
  check(mont_batch_update(b, many.data(), 4097, nullptr) == MONT_ERANGE, "count above the capacity");
  check(mont_batch_destroy(b) == MONT_OK, "destroy");
  // small capacities, exactly full
  for (int cap : {1, 2, 16, 17, 33}) {
    mont_batch* c = nullptr;
    check(mont_batch_reserve(cap, &c) == MONT_OK, "reserve");
    for (int rep = 0; rep < 4; rep++) check(run_batch(c, vs, rng, cap - rep % 2, 9000, rep & 1), "full small batch");
    check(mont_batch_destroy(c) == MONT_OK, "destroy small");
  }
  check(mont_batch_reserve(0, &b) == MONT_EINVAL, "reserve 0");
  check(hip_stub_live_allocs == 0, "every allocation freed");
  printf("%ld launches, %ld copies, %d failures\n", hip_stub_launches, hip_stub_copies, failures);
  return failures == 0 ? 0 : 1;
}
