// Sanitizer driver for the CPU oracle and the input generators (built with the
// host compiler's address and undefined-behaviour sanitizers by
// tests/test_sanitizers.py): every oracle entry point on generated ligands of
// 1 to 64 atoms and 0 to 8 rotatable bonds, both precisions, including the
// degenerate sizes (one atom, no bonds, one sample per scan, no sweeps).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

// The oracle's C interface (oracle/oracle.cpp), as its ctypes loader declares it.
extern "C" {
typedef struct { int nx, ny, nz; double origin[3]; double spacing, inv_spacing, out_value; const float* values; } og_grid;
typedef struct {
  int N, K;
  const double* xyz;
  const double* ref;
  const int32_t* ta;
  const int32_t* tb;
  const uint32_t* mask;
  const double* inv_len;
} og_ligand;
typedef struct {
  int R, A, T, S;
  const double* restarts;
  const double* angles;
  double trans_step, clash2;
  const double* center;
} og_dock;
int oracle_dock_ligand(int, const og_grid*, const og_ligand*, const og_dock*, double*, double*, double*, int16_t*,
                       double*);
int oracle_place(int, const og_ligand*, const double*, const double*, double*, double*);
int oracle_scan(int, const og_grid*, const og_ligand*, const og_dock*, int, int, const double*, const double*, double*,
                double*, double*, int*, double*);
double oracle_score(int, const og_grid*, int, int, const double*, double*, double*);
double oracle_pose_grad(const og_grid*, const og_ligand*, const double*, const double*, double*);
int oracle_pose_map(const og_ligand*, const double*, const double*, const double*, double*);
int oracle_topk(int, const double*, int, int32_t*);
double oracle_refine(int, const og_grid*, const og_ligand*, const double*, const double*, double*, int*);
int oracle_apply_move(int, const og_ligand*, const double*, const double*, const double*, double*, double*);
double oracle_move_grad(int, const og_grid*, const og_ligand*, const double*, const double*, double*);
int oracle_move_clash_free(int, const og_ligand*, const double*, double);
// generators (gen/gen.cpp)
int gen_pocket(int, double, int, int, uint64_t, const double*, float*, float*);
int gen_ligands(int, const int64_t*, uint64_t, const int32_t*, const int32_t*, const int64_t*, const int64_t*, double*,
                int32_t*, uint32_t*, int32_t*, int32_t*, int32_t*);
int gen_restarts(int, uint64_t, double, double*, float*);
int gen_angles(int, double*, float*);
}

#define EXPECT(cond, msg)                                \
  do {                                                   \
    if (!(cond)) {                                       \
      std::fprintf(stderr, "%s\n", msg);                 \
      std::exit(1);                                      \
    }                                                    \
  } while (0)

int main() {
  const int n = 24;
  const double h = 0.5, center[3] = {1.0, -2.0, 0.5};
  std::vector<float> grid((size_t)n * n * n);
  float origin[3];
  EXPECT(gen_pocket(n, h, 12, 60, 7, center, grid.data(), origin) == 0, "gen_pocket");
  og_grid G{n, n, n, {origin[0], origin[1], origin[2]}, h, 1.0 / h, 0.0, grid.data()};
  const int sizes[][2] = {{1, 0}, {2, 0}, {5, 1}, {12, 3}, {30, 6}, {64, 8}};
  int calls = 0;
  for (auto sz : sizes) {
    const int N = sz[0], Kreq = sz[1];
    const int64_t id = 1000 + N, ao = 0, bo = 0;
    std::vector<double> xyz(3 * N);
    std::vector<int32_t> parent(N), ta(Kreq + 1), tb(Kreq + 1);
    std::vector<uint32_t> mask(N);
    int32_t K = 0;
    EXPECT(gen_ligands(1, &id, 3, &N, &Kreq, &ao, &bo, xyz.data(), parent.data(), mask.data(), ta.data(), tb.data(),
                       &K) == 0, "gen_ligands");
    std::vector<double> inv(K + 1), ref(3, 0.0);
    for (int i = 0; i < N; ++i)
      for (int a = 0; a < 3; ++a) ref[a] += xyz[3 * i + a] / N;
    for (int k = 0; k < K; ++k) {
      double d2 = 0;
      for (int a = 0; a < 3; ++a) d2 += std::pow(xyz[3 * tb[k] + a] - xyz[3 * ta[k] + a], 2);
      inv[k] = 1.0 / std::sqrt(d2);
    }
    og_ligand L{N, K, xyz.data(), ref.data(), ta.data(), tb.data(), mask.data(), inv.data()};
    for (int A : {1, 16}) {
      const int R = 3, T = A;
      std::vector<double> r64(12 * R), a64(2 * A);
      std::vector<float> r32(12 * R), a32(2 * A);
      gen_restarts(R, 5, 2.0, r64.data(), r32.data());
      gen_angles(A, a64.data(), a32.data());
      for (int S : {0, 2}) {
        og_dock D{R, A, T, S, r64.data(), a64.data(), 4.0 / T, 4.84, center};
        for (int bits : {32, 64}) {
          std::vector<double> fin(R), poses(3 * N * R), piv(3 * R), ss(R * S * (6 + K) + 1);
          std::vector<int16_t> tr(R * S * (6 + K) + 1);
          oracle_dock_ligand(bits, &G, &L, &D, fin.data(), poses.data(), piv.data(), tr.data(), ss.data());
          for (double f : fin) EXPECT(std::isfinite(f), "non-finite final score");
          std::vector<int32_t> top(R);
          oracle_topk(R, fin.data(), R, top.data());
          std::vector<double> x(3 * N), P(3), xo(3 * N), Po(3), samples(A > T ? A : T);
          std::vector<int> ok(samples.size());
          double best = 0;
          oracle_place(bits, &L, r64.data() + 12, center, x.data(), P.data());
          for (int kind = 0; kind < 3; ++kind)
            for (int which = 0; which < (kind == 2 ? K : 3); ++which)
              oracle_scan(bits, &G, &L, &D, kind, which, x.data(), P.data(), xo.data(), Po.data(), samples.data(),
                          ok.data(), &best);
          std::vector<double> per(N), gr(3 * N), g(6 + K), q(6 + K, 0.05), mapped(3 * N);
          oracle_score(bits, &G, 0, N, poses.data(), per.data(), nullptr);
          oracle_score(bits, &G, 1, N, poses.data(), per.data(), gr.data());
          oracle_pose_grad(&G, &L, poses.data(), piv.data(), g.data());
          oracle_pose_map(&L, poses.data(), piv.data(), q.data(), mapped.data());
          oracle_apply_move(bits, &L, poses.data(), piv.data(), q.data(), xo.data(), Po.data());
          oracle_move_grad(bits, &G, &L, poses.data(), piv.data(), g.data());
          (void)oracle_move_clash_free(bits, &L, poses.data(), 4.84);
          const double prm[8] = {5, 1e-2, 1e-3, 1e-3, 0.1, 0.05, 0.1, 4.84};
          int acc = 0;
          L.xyz = poses.data();
          const double s = oracle_refine(bits, &G, &L, piv.data(), prm, xo.data(), &acc);
          L.xyz = xyz.data();
          EXPECT(std::isfinite(s) && acc >= 0 && acc <= 5, "refine");
          calls += 12;
        }
      }
    }
  }
  std::printf("oracle: %d entry-point calls on ligands of 1..64 atoms, no sanitizer findings\n", calls);
  return 0;
}
