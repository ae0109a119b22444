// Sanitizer driver for the library's host-side checks (built with the host
// compiler's address and undefined-behaviour sanitizers by tests/test_sanitizers.py).
// Random well-formed and malformed ligand batches, host libraries, tunings and
// host-only calls; well-formed inputs must pass, each planted defect must be
// reported, and no input may read outside its arrays or hit undefined behaviour.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <random>
#include <stdexcept>
#include <string>
#include <algorithm>
#include <vector>

#include "host_checks.h"

#define EXPECT(cond, ...)                 \
  do {                                    \
    if (!(cond)) {                        \
      std::fprintf(stderr, __VA_ARGS__);  \
      std::fprintf(stderr, "\n");         \
      std::exit(1);                       \
    }                                     \
  } while (0)

struct Batch {
  std::vector<int32_t> ao, to, ta;
  int total_atoms = 0, total_tors = 0;
};

static Batch make_batch(std::mt19937_64& rng, int n) {
  Batch b;
  b.ao.assign(n + 1, 0);
  b.to.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int N = 1 + (int)(rng() % LG_MAX_ATOMS);
    const int K = N < 2 ? 0 : (int)(rng() % (LG_MAX_TORSIONS + 1));
    b.ao[i + 1] = b.ao[i] + N;
    b.to[i + 1] = b.to[i] + K;
    for (int k = 0; k < K; ++k) {
      const int a = (int)(rng() % N);
      int c = (int)(rng() % N);
      if (c == a) c = (a + 1) % N;
      b.ta.push_back(a);
      b.ta.push_back(c);
    }
  }
  b.total_atoms = b.ao[n];
  b.total_tors = b.to[n];
  return b;
}

static lg_ligands as_device(const Batch& b, int n, const void* fake) {
  lg_ligands L;
  std::memset(&L, 0, sizeof L);
  L.n = n;
  L.total_atoms = b.total_atoms;
  L.total_torsions = b.total_tors;
  // device pointers are never dereferenced on the host: any non-null value
  L.atom_offset = L.tors_offset = L.tors_atoms = (const int32_t*)fake;
  L.x = L.y = L.z = L.inv_bond_len = L.ref_point = (const float*)fake;
  L.frag_mask = (const uint32_t*)fake;
  L.atom_offset_host = b.ao.data();
  L.tors_offset_host = b.to.data();
  L.tors_atoms_host = b.ta.empty() ? b.ao.data() : b.ta.data();
  return L;
}

int main() {
  std::mt19937_64 rng(12345);
  const int fake = 0;
  std::vector<float> fx(1 << 16, 0.f);
  std::vector<uint32_t> fm(1 << 16, 0u);
  int rejected = 0;
  for (int iter = 0; iter < 3000; ++iter) {
    const int n = 1 + (int)(rng() % 40);
    Batch b = make_batch(rng, n);
    lg_ligands L = as_device(b, n, &fake);
    EXPECT(lghost::check_ligands(&L, true) == LG_OK, "well-formed batch rejected: %s", lg_last_error());
    int ma = 0, mt = 0;
    lghost::host_maxima(&L, &ma, &mt);
    EXPECT(ma >= 1 && ma <= LG_MAX_ATOMS && mt >= 0 && mt <= LG_MAX_TORSIONS, "maxima %d %d", ma, mt);
    // one planted defect
    const int kind = (int)(rng() % 7);
    const int i = (int)(rng() % n);
    switch (kind) {
      case 0: b.ao[i + 1] = b.ao[i]; break;                                   // empty ligand
      case 1: b.ao[i + 1] = b.ao[i] + LG_MAX_ATOMS + 1 + (int)(rng() % 5); break;
      case 2: b.to[i + 1] = b.to[i] - 1 - (int)(rng() % 3); break;            // decreasing
      case 3: b.ao[n] = b.total_atoms + 1; break;                             // wrong total
      case 4: b.ao[i + 1] = (int32_t)0x7fffff00; b.ao[i] = (int32_t)-0x7fffff00; break;   // extreme values
      case 5:
        if (b.total_tors == 0) { b.to[n] = 1; break; }
        b.ta[rng() % b.ta.size()] = LG_MAX_ATOMS + 3;                         // bond id out of range
        break;
      default:
        if (b.total_tors == 0) { b.ao[0] = 1; break; }
        { const size_t k = 2 * (rng() % (size_t)b.total_tors); b.ta[k + 1] = b.ta[k]; }   // same atom twice
    }
    L = as_device(b, n, &fake);
    EXPECT(lghost::check_ligands(&L, true) != LG_OK, "defect %d not reported", kind);
    EXPECT(std::strlen(lg_last_error()) > 0, "no message");
    ++rejected;

    // the same library held on the host
    Batch h = make_batch(rng, n);
    std::vector<float> x(h.total_atoms), ref(3 * n), il(h.total_tors + 1);
    std::vector<uint32_t> mk(h.total_atoms);
    // the bond array on the heap at its exact size, so that a read past it is reported
    std::unique_ptr<int32_t[]> tab(new int32_t[h.ta.size() + 1]);
    lg_host_ligands H{n, h.total_atoms, h.total_tors, h.ao.data(), h.to.data(), x.data(), x.data(), x.data(),
                      mk.data(), tab.get(), il.data(), ref.data()};
    auto sync_bonds = [&]() { std::copy(h.ta.begin(), h.ta.end(), tab.get()); tab[h.ta.size()] = 0; };
    sync_bonds();
    EXPECT(lghost::check_host_ligands(&H) == LG_OK, "well-formed host library rejected: %s", lg_last_error());
    const int j = (int)(rng() % n);
    switch (rng() % 3) {
      case 0:   // a ligand's bond range runs past the next one's (ends beyond the array for the last pair)
        if (j + 2 <= n) { h.to[j + 1] = h.to[j + 2] + 1; break; }
        h.ao[n] += 1;
        break;
      case 1: h.ao[j + 1] = h.ao[j]; break;
      default:
        if (h.total_tors == 0) { h.to[0] = -1; break; }
        { const size_t k = 2 * (rng() % (size_t)h.total_tors); h.ta[k] = (rng() & 1) ? h.ta[k + 1] : -1; }
    }
    sync_bonds();
    EXPECT(lghost::check_host_ligands(&H) != LG_OK, "host library defect not reported");
  }
  // tunings: random fields, accepted exactly when every field is in range
  for (int iter = 0; iter < 20000; ++iter) {
    lg_tuning t;
    std::memset(&t, 0, sizeof t);
    t.n_atom_clusters = (int)(rng() % 18) - 1;
    t.n_rot_clusters = (int)(rng() % 34) - 1;
    for (int c = 0; c < 16; ++c) t.atom_bounds[c] = 16 * (c + 1) + (int)(rng() % 3) - 1;
    for (int c = 0; c < 32; ++c) t.rot_bounds[c] = c + (int)(rng() % 2);
    for (int c = 0; c < 4; ++c) t.waves_per_block[c] = 1 << (int)(rng() % 3);
    t.restart_chunk = (rng() % 50 == 0) ? (int)(rng() % 200000) - 10 : 1 + (int)(rng() % 64);
    t.grid_scale = (int)(rng() % 70) - 2;
    t.plain_waves_per_block = 1 << (int)(rng() % 3);
    t.use_graph = (int)(rng() % 3);
    t.lazy_clash = (int)(rng() % 2);
    (void)lghost::check_tuning(&t);
  }
  // host-only calls over their argument ranges
  int32_t bounds[64];
  for (int nc = -2; nc < 40; ++nc)
    for (int mx = -2; mx < 300; mx += 7) {
      const int a = lg_atom_clusters(nc, 64, mx, bounds);
      EXPECT(a >= 0 && a <= (nc > 0 ? nc : 0), "atom clusters %d", a);
      const int r = lg_rotamer_clusters(nc, mx, bounds);
      EXPECT(r >= 0 && r <= (nc > 0 ? nc : 0), "rotamer clusters %d", r);
      for (int c = 1; c < r; ++c) EXPECT(bounds[c] > bounds[c - 1], "rotamer bounds not increasing");
    }
  EXPECT(lg_bucket_size(16, 108, 32, 32) == 1728, "Eq. 1");
  EXPECT(lg_bucket_size(1, 1, 0, 64) == -1, "Eq. 1 bad args");
  EXPECT(lghost::check_ligands(nullptr, true) == LG_ERR_INVALID_ARG, "null batch");
  // the error message lives in a fixed buffer: a longer one is cut, terminated
  std::string long_msg(2000, 'm');
  EXPECT(lghost::fail(LG_ERR_LIMIT, "%s", long_msg.c_str()) == LG_ERR_LIMIT, "fail returns its status");
  EXPECT(std::strlen(lg_last_error()) == 511 && lg_last_error()[0] == 'm', "long message not cut at 511");
  EXPECT(lghost::fail(LG_ERR_INVALID_ARG, "short %d", 7) == LG_ERR_INVALID_ARG &&
         std::strcmp(lg_last_error(), "short 7") == 0, "short message after a long one");
  // the stream unpack's slices tile every copy in order, starts page-aligned
  for (size_t bytes : {(size_t)0, (size_t)4, (size_t)4096, (size_t)4100, (size_t)1 << 20, ((size_t)3 << 20) + 77,
                       (size_t)123456789, (size_t)1 << 33})
    for (int slices = 1; slices <= 8; ++slices) {
      size_t pos = 0;
      for (int s = 0; s < slices; ++s) {
        size_t b0, b1;
        lghost::copy_slice(bytes, slices, s, &b0, &b1);
        EXPECT(b0 <= b1 && (b0 == pos || b0 == b1), "slice %d/%d of %zu: [%zu, %zu) after %zu", s, slices, bytes, b0, b1, pos);
        EXPECT(b0 == b1 || b0 % 4096 == 0 || s == 0, "slice start not page-aligned");
        if (b1 > b0) pos = b1;
      }
      EXPECT(pos == bytes, "slices of %zu bytes end at %zu", bytes, pos);
    }
  // exceptions stop at the boundary as status codes, results pass through
  EXPECT(lghost::guarded([] { return LG_ERR_LIMIT; }) == LG_ERR_LIMIT, "guarded result");
  EXPECT(lghost::guarded([]() -> lg_status { throw std::bad_alloc(); }) == LG_ERR_OUT_OF_MEMORY &&
         std::strstr(lg_last_error(), "host memory") != nullptr, "bad_alloc not mapped");
  EXPECT(lghost::guarded([]() -> lg_status { throw std::runtime_error("thread start"); }) == LG_ERR_DEVICE &&
         std::strstr(lg_last_error(), "thread start") != nullptr, "exception not mapped");
  EXPECT(lghost::guarded([]() -> lg_status { throw 3; }) == LG_ERR_DEVICE, "non-exception throw not mapped");
  std::printf("host checks: %d planted defects reported, no sanitizer findings\n", rejected);
  return 0;
}
