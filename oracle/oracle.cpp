// CPU ORACLE for the docking hot path -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
// load this library.  The product path (the HIP library) never calls it and
// shares no code, header or table with it.
//
// Plain, single-threaded, slow on purpose.  Every routine is a template on the
// arithmetic type R:
//   R = float  reproduces the FP32 arithmetic contract bit for bit (explicit
//              fma, no contraction, sums in atom order), used for index, pose
//              and score parity with the GPU;
//   R = double is used for invariants and finite differences.
//
// What the method computes.  The paper (Sec. 2) states the problem: dock each
// ligand of a chemical library into a docking site, i.e. estimate the 3D
// placement of its atoms, then score the interaction and rank the library.
// Its cost grows with the number of atoms and of rotamers (rotatable
// fragments, Sec. 3).  The paper does not print LiGen's search or scoring
// function; the steps below are this project's reading of that statement:
//   restart placement -> S sweeps of {rigid rotation scans about x,y,z;
//   rigid translation scans along x,y,z; greedy torsion scans with an
//   intramolecular clash check} scored by nearest-voxel grid lookups ->
//   trilinear final score -> per-ligand top-k over restarts.
// Each helper names the step it implements.  Sample j = 0 of every scan is the
// current pose itself (identity move): always admissible, and selecting it
// leaves the pose untouched, so every restart's scan score never decreases.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

extern "C" {
typedef struct {
  int nx, ny, nz;
  double origin[3];
  double spacing, inv_spacing, out_value;
  const float* values;      // [nz][ny][nx], x fastest
} og_grid;

typedef struct {
  int N, K;
  const double* xyz;        // [N][3] input conformation
  const double* ref;        // [3] pivot P0
  const int32_t* ta;        // [K] static-side pivot atom a_k
  const int32_t* tb;        // [K] moving-side atom b_k
  const uint32_t* mask;     // [N] bit k: atom moves with bond k (fragment F_k, contains b_k)
  const double* inv_len;    // [K] 1 / |x_b - x_a| of the input
} og_ligand;

typedef struct {
  int R, A, T, S;
  const double* restarts;   // [R][12] row-major rotation, then offset
  const double* angles;     // [A][2] (cos, sin) of 2*pi*j/A
  double trans_step;        // delta: offset of translation sample j is delta*(j<T/2 ? j : j-T)
  double clash2;            // squared clash distance
  const double* center;     // [3] pocket centre
} og_dock;
}

namespace {

template <class R>
struct Grid {
  int n[3];
  R o[3], h, inv_h, out;
  R c0[3];    // offset of the nearest-node map: c0 = fma(-o, 1/h, 1/2)
  const float* v;
  explicit Grid(const og_grid* g) : h((R)g->spacing), inv_h((R)g->inv_spacing), out((R)g->out_value), v(g->values) {
    n[0] = g->nx; n[1] = g->ny; n[2] = g->nz;
    for (int a = 0; a < 3; ++a) {
      o[a] = (R)g->origin[a];
      c0[a] = std::fma(-o[a], inv_h, (R)0.5);
    }
  }
  R at(int ix, int iy, int iz) const { return (R)v[((size_t)iz * n[1] + iy) * n[0] + ix]; }
};

template <class R>
struct Lig {
  int N, K;
  std::vector<R> x0[3];
  R P0[3];
  std::vector<int> ta, tb;
  std::vector<uint32_t> mask;
  std::vector<R> inv_len;
  explicit Lig(const og_ligand* l) : N(l->N), K(l->K), ta(l->ta, l->ta + l->K), tb(l->tb, l->tb + l->K),
                                      mask(l->mask, l->mask + l->N), inv_len(l->K) {
    for (int a = 0; a < 3; ++a) {
      x0[a].resize(N);
      for (int i = 0; i < N; ++i) x0[a][i] = (R)l->xyz[3 * i + a];
      P0[a] = (R)l->ref[a];
    }
    for (int k = 0; k < K; ++k) inv_len[k] = (R)l->inv_len[k];
  }
  bool moves(int i, int k) const { return (mask[i] >> k) & 1u; }
};

template <class R>
struct Pose {
  std::vector<R> X[3];   // coordinates per axis
  R P[3];                // rigid-body pivot
  explicit Pose(int N = 0) { for (auto& a : X) a.assign(N, (R)0); P[0] = P[1] = P[2] = (R)0; }
};

using std::fma;

// ---- nearest-voxel lookup: the nearest node of coordinate x is round((x - o)/h),
// evaluated per axis as the affine map f = fma(x, 1/h, c0) with
// c0 = fma(-o, 1/h, 1/2); the atom is in the grid iff 0 <= f < n on every axis,
// then the node is (int)f; otherwise it contributes the far-field value.
template <class R>
R nearest(const Grid<R>& g, R x, R y, R z) {
  R c[3] = {x, y, z};
  int i[3];
  for (int a = 0; a < 3; ++a) {
    R f = fma(c[a], g.inv_h, g.c0[a]);
    if (!(f >= (R)0 && f < (R)g.n[a])) return g.out;
    i[a] = (int)f;
  }
  return g.at(i[0], i[1], i[2]);
}

// ---- pose score during the scans: sum of nearest values, in atom order.
template <class R>
R score_nearest(const Grid<R>& g, const Pose<R>& p) {
  R s = (R)0;
  for (size_t i = 0; i < p.X[0].size(); ++i) s = s + nearest(g, p.X[0][i], p.X[1][i], p.X[2][i]);
  return s;
}

// ---- trilinear value and gradient: f = (x - o)/h per axis; in range iff
// 0 <= f < n-1 on every axis, else the far-field value with zero gradient.
// Corner values lerp along x, then y, then z, each lerp as fma(w, hi-lo, lo).
template <class R>
R trilinear(const Grid<R>& g, R x, R y, R z, R* grad) {
  R c[3] = {x, y, z}, f[3], w[3];
  int i[3];
  for (int a = 0; a < 3; ++a) {
    f[a] = (c[a] - g.o[a]) * g.inv_h;
    if (!(f[a] >= (R)0 && f[a] < (R)(g.n[a] - 1))) {
      if (grad) grad[0] = grad[1] = grad[2] = (R)0;
      return g.out;
    }
    i[a] = (int)f[a];
    w[a] = f[a] - (R)i[a];
  }
  R c000 = g.at(i[0], i[1], i[2]), c100 = g.at(i[0] + 1, i[1], i[2]);
  R c010 = g.at(i[0], i[1] + 1, i[2]), c110 = g.at(i[0] + 1, i[1] + 1, i[2]);
  R c001 = g.at(i[0], i[1], i[2] + 1), c101 = g.at(i[0] + 1, i[1], i[2] + 1);
  R c011 = g.at(i[0], i[1] + 1, i[2] + 1), c111 = g.at(i[0] + 1, i[1] + 1, i[2] + 1);
  R c00 = fma(w[0], c100 - c000, c000), c10 = fma(w[0], c110 - c010, c010);
  R c01 = fma(w[0], c101 - c001, c001), c11 = fma(w[0], c111 - c011, c011);
  R c0 = fma(w[1], c10 - c00, c00), c1 = fma(w[1], c11 - c01, c01);
  R v = fma(w[2], c1 - c0, c0);
  if (grad) {
    R e00 = c100 - c000, e10 = c110 - c010, e01 = c101 - c001, e11 = c111 - c011;
    R e0 = fma(w[1], e10 - e00, e00), e1 = fma(w[1], e11 - e01, e01);
    grad[0] = fma(w[2], e1 - e0, e0) * g.inv_h;
    R d0 = c10 - c00, d1 = c11 - c01;
    grad[1] = fma(w[2], d1 - d0, d0) * g.inv_h;
    grad[2] = (c1 - c0) * g.inv_h;
  }
  return v;
}

template <class R>
R score_trilinear(const Grid<R>& g, const Pose<R>& p) {
  R s = (R)0;
  for (size_t i = 0; i < p.X[0].size(); ++i) s = s + trilinear(g, p.X[0][i], p.X[1][i], p.X[2][i], (R*)nullptr);
  return s;
}

// ---- restart placement: x = M_r (x0 - P0) + (c + t_r); the pivot becomes c + t_r.
template <class R>
void place(const Lig<R>& L, const R* row, const R* center, Pose<R>& p) {
  R q[3] = {center[0] + row[9], center[1] + row[10], center[2] + row[11]};
  for (int i = 0; i < L.N; ++i) {
    R v[3] = {L.x0[0][i] - L.P0[0], L.x0[1][i] - L.P0[1], L.x0[2][i] - L.P0[2]};
    for (int a = 0; a < 3; ++a) {
      R y = fma(row[3 * a + 2], v[2], fma(row[3 * a + 1], v[1], row[3 * a] * v[0]));
      p.X[a][i] = y + q[a];
    }
  }
  for (int a = 0; a < 3; ++a) p.P[a] = q[a];
}

// ---- rigid rotation by (c, s) about the lab axis e through the pivot.
// The two other axes (p, q) follow cyclically: e=x -> (y,z), y -> (z,x), z -> (x,y).
template <class R>
void rotate_lab(const Pose<R>& in, int e, R c, R s, Pose<R>& out) {
  int p = (e + 1) % 3, q = (e + 2) % 3;
  out = in;
  for (size_t i = 0; i < in.X[0].size(); ++i) {
    R vp = in.X[p][i] - in.P[p], vq = in.X[q][i] - in.P[q];
    R np = fma(c, vp, -(s * vq));
    R nq = fma(s, vp, c * vq);
    out.X[p][i] = in.P[p] + np;
    out.X[q][i] = in.P[q] + nq;
  }
}

// ---- rigid translation along lab axis e by d (the pivot moves along).
template <class R>
void translate(const Pose<R>& in, int e, R d, Pose<R>& out) {
  out = in;
  for (size_t i = 0; i < in.X[0].size(); ++i) out.X[e][i] = in.X[e][i] + d;
  out.P[e] = in.P[e] + d;
}

template <class R>
R translation_offset(R delta, int j, int T) {
  int m = j < T / 2 ? j : j - T;
  return delta * (R)m;
}

// ---- torsion k: rotate the moving fragment F_k minus its axis atom b_k by
// (c, s) about the bond axis a_k -> b_k (right-handed).  u = (x_b - x_a)/|bond|,
// with 1/|bond| taken from the input conformation; matrix
// M = c I + (1-c) u u^T + s [u]_x.  a_k and b_k are never transformed.
template <class R>
void torsion_matrix(R ux, R uy, R uz, R c, R s, R m[9]) {
  R t = (R)1 - c;
  R tx = t * ux, ty = t * uy, tz = t * uz;
  m[0] = fma(tx, ux, c);
  m[4] = fma(ty, uy, c);
  m[8] = fma(tz, uz, c);
  m[1] = fma(tx, uy, -(s * uz));
  m[3] = fma(tx, uy, s * uz);
  m[2] = fma(tx, uz, s * uy);
  m[6] = fma(tx, uz, -(s * uy));
  m[5] = fma(ty, uz, -(s * ux));
  m[7] = fma(ty, uz, s * ux);
}

template <class R>
void rotate_torsion(const Lig<R>& L, const Pose<R>& in, int k, R c, R s, Pose<R>& out) {
  int a = L.ta[k], b = L.tb[k];
  R u[3];
  for (int d = 0; d < 3; ++d) u[d] = (in.X[d][b] - in.X[d][a]) * L.inv_len[k];
  R m[9];
  torsion_matrix(u[0], u[1], u[2], c, s, m);
  out = in;
  for (int i = 0; i < L.N; ++i) {
    if (!L.moves(i, k) || i == b) continue;
    R v[3] = {in.X[0][i] - in.X[0][a], in.X[1][i] - in.X[1][a], in.X[2][i] - in.X[2][a]};
    for (int d = 0; d < 3; ++d) {
      R y = fma(m[3 * d + 2], v[2], fma(m[3 * d + 1], v[1], m[3 * d] * v[0]));
      out.X[d][i] = in.X[d][a] + y;
    }
  }
}

// ---- intramolecular clash check for torsion k: every pair (i, s) whose
// distance the torsion can change -- i in F_k minus b_k, s outside F_k and not
// a_k -- must satisfy d^2 >= clash2, with d^2 = fma(dz,dz, fma(dy,dy, dx*dx)).
template <class R>
bool clash_free(const Lig<R>& L, const Pose<R>& p, int k, R clash2) {
  int a = L.ta[k], b = L.tb[k];
  for (int i = 0; i < L.N; ++i) {
    if (!L.moves(i, k) || i == b) continue;
    for (int s = 0; s < L.N; ++s) {
      if (L.moves(s, k) || s == a) continue;
      R dx = p.X[0][i] - p.X[0][s], dy = p.X[1][i] - p.X[1][s], dz = p.X[2][i] - p.X[2][s];
      R d2 = fma(dz, dz, fma(dy, dy, dx * dx));
      if (d2 < clash2) return false;
    }
  }
  return true;
}

template <class R>
struct Ctx {
  Grid<R> g;
  Lig<R> L;
  int R_, A, T, S;
  std::vector<R> restarts, angles, center;
  R delta, clash2;
  Ctx(const og_grid* gg, const og_ligand* l, const og_dock* d)
      : g(gg), L(l), R_(d ? d->R : 0), A(d ? d->A : 0), T(d ? d->T : 0), S(d ? d->S : 0),
        delta(d ? (R)d->trans_step : (R)0), clash2(d ? (R)d->clash2 : (R)0) {
    if (!d) return;
    restarts.resize((size_t)R_ * 12);
    for (size_t i = 0; i < restarts.size(); ++i) restarts[i] = (R)d->restarts[i];
    angles.resize((size_t)A * 2);
    for (size_t i = 0; i < angles.size(); ++i) angles[i] = (R)d->angles[i];
    center = {(R)d->center[0], (R)d->center[1], (R)d->center[2]};
  }
};

// Scan kinds: 0 rotation about lab axis `which`, 1 translation along `which`,
// 2 torsion `which`.  Evaluates every sample, takes the best admissible one
// (strictly greater score wins, so equal scores keep the lowest index) and
// applies it.  Returns j*; fills per-sample scores / admissibility if asked.
template <class R>
int scan(const Ctx<R>& C, int kind, int which, Pose<R>& pose, R* best_score_out,
         R* sample_scores, int* sample_ok) {
  int n = kind == 1 ? C.T : C.A;
  R best = -std::numeric_limits<R>::infinity();
  int jbest = -1;
  Pose<R> cand(C.L.N);
  Pose<R> chosen = pose;
  for (int j = 0; j < n; ++j) {
    bool ok = true;
    if (j == 0) {
      cand = pose;
    } else if (kind == 0) {
      rotate_lab(pose, which, C.angles[2 * j], C.angles[2 * j + 1], cand);
    } else if (kind == 1) {
      translate(pose, which, translation_offset(C.delta, j, C.T), cand);
    } else {
      rotate_torsion(C.L, pose, which, C.angles[2 * j], C.angles[2 * j + 1], cand);
      ok = clash_free(C.L, cand, which, C.clash2);
    }
    R sc = score_nearest(C.g, cand);
    if (sample_scores) sample_scores[j] = sc;
    if (sample_ok) sample_ok[j] = ok ? 1 : 0;
    if (ok && sc > best) { best = sc; jbest = j; chosen = cand; }
  }
  pose = chosen;
  if (best_score_out) *best_score_out = best;
  return jbest;
}

// One restart: placement, S sweeps, final trilinear score.
template <class R>
R dock_restart(const Ctx<R>& C, int r, Pose<R>& pose, int16_t* trace, R* scan_scores) {
  place(C.L, &C.restarts[(size_t)r * 12], C.center.data(), pose);
  int per = 6 + C.L.K, t = 0;
  for (int s = 0; s < C.S; ++s) {
    for (int e = 0; e < 3; ++e, ++t) {
      R b; int j = scan(C, 0, e, pose, &b, (R*)nullptr, (int*)nullptr);
      if (trace) trace[s * per + e] = (int16_t)j;
      if (scan_scores) scan_scores[s * per + e] = b;
    }
    for (int e = 0; e < 3; ++e) {
      R b; int j = scan(C, 1, e, pose, &b, (R*)nullptr, (int*)nullptr);
      if (trace) trace[s * per + 3 + e] = (int16_t)j;
      if (scan_scores) scan_scores[s * per + 3 + e] = b;
    }
    for (int k = 0; k < C.L.K; ++k) {
      R b; int j = scan(C, 2, k, pose, &b, (R*)nullptr, (int*)nullptr);
      if (trace) trace[s * per + 6 + k] = (int16_t)j;
      if (scan_scores) scan_scores[s * per + 6 + k] = b;
    }
  }
  (void)t;
  return score_trilinear(C.g, pose);
}

template <class R>
void to_pose(const Lig<R>& L, const double* xyz, const double* P, Pose<R>& p) {
  p = Pose<R>(L.N);
  for (int i = 0; i < L.N; ++i)
    for (int a = 0; a < 3; ++a) p.X[a][i] = (R)xyz[3 * i + a];
  for (int a = 0; a < 3; ++a) p.P[a] = P ? (R)P[a] : (R)0;
}

template <class R>
void from_pose(const Pose<R>& p, double* xyz, double* P) {
  size_t N = p.X[0].size();
  if (xyz)
    for (size_t i = 0; i < N; ++i)
      for (int a = 0; a < 3; ++a) xyz[3 * i + a] = (double)p.X[a][i];
  if (P) for (int a = 0; a < 3; ++a) P[a] = (double)p.P[a];
}

template <class R>
int dock_ligand(const og_grid* g, const og_ligand* l, const og_dock* d, double* final_scores,
                double* poses, double* pivots, int16_t* trace, double* scan_scores) {
  Ctx<R> C(g, l, d);
  int per = d->S * (6 + l->K);
  std::vector<R> ss(per);
  for (int r = 0; r < d->R; ++r) {
    Pose<R> p(l->N);
    R f = dock_restart(C, r, p, trace ? trace + (size_t)r * per : nullptr, scan_scores ? ss.data() : nullptr);
    final_scores[r] = (double)f;
    if (poses) from_pose(p, poses + (size_t)r * l->N * 3, (double*)nullptr);
    if (pivots) for (int a = 0; a < 3; ++a) pivots[3 * r + a] = (double)p.P[a];
    if (scan_scores) for (int i = 0; i < per; ++i) scan_scores[(size_t)r * per + i] = (double)ss[i];
  }
  return 0;
}

// ---- refinement pose map (FP64 definition used for the adjoint check):
// torsions in reverse bond order (k = K-1 .. 0; deepest first for parents-first
// bond lists) about the current bond axes, then a rotation Exp(omega) about the
// pivot, then + t.
void rodrigues(const double u[3], double th, double m[9]) {
  double c = std::cos(th), s = std::sin(th), t = 1 - c;
  m[0] = c + t * u[0] * u[0];        m[1] = t * u[0] * u[1] - s * u[2]; m[2] = t * u[0] * u[2] + s * u[1];
  m[3] = t * u[0] * u[1] + s * u[2]; m[4] = c + t * u[1] * u[1];        m[5] = t * u[1] * u[2] - s * u[0];
  m[6] = t * u[0] * u[2] - s * u[1]; m[7] = t * u[1] * u[2] + s * u[0]; m[8] = c + t * u[2] * u[2];
}

// ---- (cos x, sin x) of a refinement step angle.  Steps are clipped to at most
// pi/4, where the Taylor series to x^13 / x^12 (Horner in x^2, fma) is accurate to
// well below an FP32 ulp; the same polynomial is the arithmetic contract of
// refinement in both precisions.  Larger angles (only reachable through
// apply_move called directly) use the library functions.
template <class R>
void step_cos_sin(R x, R& c, R& s) {
  if (!(std::fabs(x) <= (R)0.7853981633974483)) {
    c = std::cos(x);
    s = std::sin(x);
    return;
  }
  const R x2 = x * x;
  R ps = (R)(1.0 / 6227020800.0);
  ps = fma(ps, x2, (R)(-1.0 / 39916800.0));
  ps = fma(ps, x2, (R)(1.0 / 362880.0));
  ps = fma(ps, x2, (R)(-1.0 / 5040.0));
  ps = fma(ps, x2, (R)(1.0 / 120.0));
  ps = fma(ps, x2, (R)(-1.0 / 6.0));
  s = fma(x * x2, ps, x);
  R pc = (R)(1.0 / 479001600.0);
  pc = fma(pc, x2, (R)(-1.0 / 3628800.0));
  pc = fma(pc, x2, (R)(1.0 / 40320.0));
  pc = fma(pc, x2, (R)(-1.0 / 720.0));
  pc = fma(pc, x2, (R)(1.0 / 24.0));
  pc = fma(pc, x2, (R)(-0.5));
  c = fma(x2, pc, (R)1);
}

// ---- local move (t, omega, theta) applied to a pose: torsions in reverse bond order
// (k = K-1 .. 0) about the current bond axes, then the rotation by |omega|
// about the axis omega/|omega| through the pivot, then + t (the pivot moves
// with t).  Every rotation uses the torsion-scan matrix script with the
// (cos, sin) of its angle; torsion axes are (x_b - x_a) * inv_len as in the scans.
template <class R>
void apply_move(const Lig<R>& L, Pose<R>& p, const R* q) {
  for (int k = L.K - 1; k >= 0; --k) {
    const R th = q[6 + k];
    if (th == (R)0) continue;
    R c, sn;
    step_cos_sin(th, c, sn);
    rotate_torsion(L, p, k, c, sn, p);
  }
  const R w2 = fma(q[5], q[5], fma(q[4], q[4], q[3] * q[3]));
  if (w2 > (R)0) {
    const R w = std::sqrt(w2);
    R m[9], c, sn;
    step_cos_sin(w, c, sn);
    torsion_matrix(q[3] / w, q[4] / w, q[5] / w, c, sn, m);
    for (size_t i = 0; i < p.X[0].size(); ++i) {
      R v[3] = {p.X[0][i] - p.P[0], p.X[1][i] - p.P[1], p.X[2][i] - p.P[2]};
      for (int d = 0; d < 3; ++d) {
        R y = fma(m[3 * d + 2], v[2], fma(m[3 * d + 1], v[1], m[3 * d] * v[0]));
        p.X[d][i] = p.P[d] + y;
      }
    }
  }
  for (int d = 0; d < 3; ++d) {
    for (size_t i = 0; i < p.X[0].size(); ++i) p.X[d][i] = p.X[d][i] + q[d];
    p.P[d] = p.P[d] + q[d];
  }
}

// ---- trilinear score of a pose and its gradient with respect to the local
// move at zero (force / torque form, torsion axes (x_b - x_a) * inv_len); sums
// in atom order.
template <class R>
R move_gradient(const Grid<R>& g, const Lig<R>& L, const Pose<R>& p, std::vector<R>& grad) {
  const int N = L.N, K = L.K;
  std::vector<R> ga((size_t)3 * N);
  R s = (R)0;
  for (int i = 0; i < N; ++i) s = s + trilinear(g, p.X[0][i], p.X[1][i], p.X[2][i], &ga[3 * i]);
  grad.assign(6 + K, (R)0);
  for (int i = 0; i < N; ++i) {
    const R* gi = &ga[3 * i];
    R r[3] = {p.X[0][i] - p.P[0], p.X[1][i] - p.P[1], p.X[2][i] - p.P[2]};
    for (int d = 0; d < 3; ++d) grad[d] = grad[d] + gi[d];
    grad[3] = grad[3] + (r[1] * gi[2] - r[2] * gi[1]);
    grad[4] = grad[4] + (r[2] * gi[0] - r[0] * gi[2]);
    grad[5] = grad[5] + (r[0] * gi[1] - r[1] * gi[0]);
  }
  for (int k = 0; k < K; ++k) {
    const int a = L.ta[k], b = L.tb[k];
    R u[3];
    for (int d = 0; d < 3; ++d) u[d] = (p.X[d][b] - p.X[d][a]) * L.inv_len[k];
    R t[3] = {(R)0, (R)0, (R)0};
    for (int i = 0; i < N; ++i) {
      if (!L.moves(i, k)) continue;
      const R* gi = &ga[3 * i];
      R r[3] = {p.X[0][i] - p.X[0][a], p.X[1][i] - p.X[1][a], p.X[2][i] - p.X[2][a]};
      t[0] = t[0] + (r[1] * gi[2] - r[2] * gi[1]);
      t[1] = t[1] + (r[2] * gi[0] - r[0] * gi[2]);
      t[2] = t[2] + (r[0] * gi[1] - r[1] * gi[0]);
    }
    grad[6 + k] = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
  }
  return s;
}

// ---- intramolecular clash rule of refinement: the union over bonds of the
// pairs a torsion can move -- (i, j) such that for some bond k exactly one of
// them is in F_k, the moving one is not b_k and the other is not a_k -- must all
// satisfy d^2 >= clash2.
template <class R>
bool move_clash_free(const Lig<R>& L, const Pose<R>& p, R clash2) {
  for (int i = 0; i < L.N; ++i)
    for (int j = i + 1; j < L.N; ++j) {
      uint32_t diff = L.mask[i] ^ L.mask[j];
      bool changes = false;
      for (int k = 0; k < L.K && !changes; ++k) {
        if (!((diff >> k) & 1u)) continue;
        const int mover = L.moves(i, k) ? i : j, other = mover == i ? j : i;
        changes = mover != L.tb[k] && other != L.ta[k];
      }
      if (!changes) continue;
      R dx = p.X[0][i] - p.X[0][j], dy = p.X[1][i] - p.X[1][j], dz = p.X[2][i] - p.X[2][j];
      if (fma(dz, dz, fma(dy, dy, dx * dx)) < clash2) return false;
    }
  return true;
}

// ---- local refinement: `steps` gradient-ascent steps on the trilinear score.
// Step = (eta_t g_t, eta_w g_w, eta_th g_th) with g_t and g_w clipped to norms
// clip_t and clip_w and every g_th component to [-clip_th, clip_th], times the
// current step scale (initially 1).  A step whose pose breaks the clash rule is
// rejected (pose kept) and halves the step scale.  The best-scoring pose seen,
// the input included, is returned.
template <class R>
struct RefineP {
  int steps;
  R eta_t, eta_w, eta_th, clip_t, clip_w, clip_th, clash2;
};

template <class R>
R refine(const Grid<R>& g, const Lig<R>& L, Pose<R>& pose, const RefineP<R>& rp, int* accepted) {
  Pose<R> best = pose;
  R best_s = score_trilinear(g, pose);
  R scale = (R)1;
  int acc = 0;
  std::vector<R> grad, q(6 + L.K);
  for (int step = 0; step < rp.steps; ++step) {
    move_gradient(g, L, pose, grad);
    R dt[3], dw[3];
    for (int d = 0; d < 3; ++d) { dt[d] = rp.eta_t * grad[d]; dw[d] = rp.eta_w * grad[3 + d]; }
    const R nt = std::sqrt(fma(dt[2], dt[2], fma(dt[1], dt[1], dt[0] * dt[0])));
    const R nw = std::sqrt(fma(dw[2], dw[2], fma(dw[1], dw[1], dw[0] * dw[0])));
    const R ft = nt > rp.clip_t ? rp.clip_t / nt : (R)1;
    const R fw = nw > rp.clip_w ? rp.clip_w / nw : (R)1;
    for (int d = 0; d < 3; ++d) {
      q[d] = (dt[d] * ft) * scale;
      q[3 + d] = (dw[d] * fw) * scale;
    }
    for (int k = 0; k < L.K; ++k) {
      R v = rp.eta_th * grad[6 + k];
      v = std::min(std::max(v, -rp.clip_th), rp.clip_th);
      q[6 + k] = v * scale;
    }
    Pose<R> cand = pose;
    apply_move(L, cand, q.data());
    if (!move_clash_free(L, cand, rp.clash2)) {
      scale = scale * (R)0.5;
      continue;
    }
    pose = cand;
    ++acc;
    const R s = score_trilinear(g, pose);
    if (s > best_s) { best_s = s; best = pose; }
  }
  pose = best;
  if (accepted) *accepted = acc;
  return best_s;
}

template <class R>
double refine_t(const og_grid* gg, const og_ligand* l, const double* P, const double* prm, double* out_xyz,
                int* accepted) {
  Grid<R> g(gg);
  Lig<R> L(l);
  Pose<R> p;
  to_pose(L, l->xyz, P, p);
  RefineP<R> rp{(int)prm[0], (R)prm[1], (R)prm[2], (R)prm[3], (R)prm[4], (R)prm[5], (R)prm[6], (R)prm[7]};
  R s = refine(g, L, p, rp, accepted);
  from_pose(p, out_xyz, (double*)nullptr);
  return (double)s;
}

template <class R>
int apply_move_t(const og_ligand* l, const double* xyz, const double* P, const double* q, double* out_xyz,
                 double* out_P) {
  Lig<R> L(l);
  Pose<R> p;
  to_pose(L, xyz, P, p);
  std::vector<R> qq(6 + L.K);
  for (int i = 0; i < 6 + L.K; ++i) qq[i] = (R)q[i];
  apply_move(L, p, qq.data());
  from_pose(p, out_xyz, out_P);
  return 0;
}

template <class R>
double move_grad_t(const og_grid* gg, const og_ligand* l, const double* xyz, const double* P, double* grad) {
  Grid<R> g(gg);
  Lig<R> L(l);
  Pose<R> p;
  to_pose(L, xyz, P, p);
  std::vector<R> gr;
  R s = move_gradient(g, L, p, gr);
  for (int i = 0; i < 6 + L.K; ++i) grad[i] = (double)gr[i];
  return (double)s;
}

template <class R>
int move_clash_free_t(const og_ligand* l, const double* xyz, double clash2) {
  Lig<R> L(l);
  Pose<R> p;
  to_pose(L, xyz, (const double*)nullptr, p);
  return move_clash_free(L, p, (R)clash2) ? 1 : 0;
}

}  // namespace

// Dock one ligand: all restarts; final trilinear score per restart; optional
// final poses [R][N][3] and their pivots [R][3], trace of selected indices
// [R][S][6+K] and best scan score per scan [R][S][6+K].
extern "C" int oracle_dock_ligand(int real_bits, const og_grid* g, const og_ligand* l, const og_dock* d,
                       double* final_scores, double* poses, double* pivots, int16_t* trace, double* scan_scores) {
  return real_bits == 32 ? dock_ligand<float>(g, l, d, final_scores, poses, pivots, trace, scan_scores)
                         : dock_ligand<double>(g, l, d, final_scores, poses, pivots, trace, scan_scores);
}

template <class R>
static int place_t(const og_ligand* l, const double* row, const double* center, double* xyz, double* P) {
  Lig<R> L(l);
  R rr[12], c[3];
  for (int i = 0; i < 12; ++i) rr[i] = (R)row[i];
  for (int i = 0; i < 3; ++i) c[i] = (R)center[i];
  Pose<R> p(L.N);
  place(L, rr, c, p);
  from_pose(p, xyz, P);
  return 0;
}

extern "C" int oracle_place(int real_bits, const og_ligand* l, const double* row, const double* center, double* xyz, double* P) {
  return real_bits == 32 ? place_t<float>(l, row, center, xyz, P) : place_t<double>(l, row, center, xyz, P);
}

template <class R>
static int scan_t(const og_grid* g, const og_ligand* l, const og_dock* d, int kind, int which,
                  const double* xyz_in, const double* P_in, double* xyz_out, double* P_out,
                  double* sample_scores, int* sample_ok, double* best) {
  Ctx<R> C(g, l, d);
  Pose<R> p;
  to_pose(C.L, xyz_in, P_in, p);
  int n = kind == 1 ? d->T : d->A;
  std::vector<R> sc(n);
  R b;
  int j = scan(C, kind, which, p, &b, sc.data(), sample_ok);
  from_pose(p, xyz_out, P_out);
  if (sample_scores) for (int i = 0; i < n; ++i) sample_scores[i] = (double)sc[i];
  if (best) *best = (double)b;
  return j;
}

extern "C" int oracle_scan(int real_bits, const og_grid* g, const og_ligand* l, const og_dock* d, int kind, int which,
                const double* xyz_in, const double* P_in, double* xyz_out, double* P_out,
                double* sample_scores, int* sample_ok, double* best) {
  return real_bits == 32 ? scan_t<float>(g, l, d, kind, which, xyz_in, P_in, xyz_out, P_out, sample_scores, sample_ok, best)
                         : scan_t<double>(g, l, d, kind, which, xyz_in, P_in, xyz_out, P_out, sample_scores, sample_ok, best);
}

// Score of N atoms: interp 0 nearest, 1 trilinear; sum in atom order.
// Optional per-atom values [N] and trilinear gradients [N][3].
template <class R>
static double score_t(const og_grid* gg, int interp, int N, const double* xyz, double* per_atom, double* grad) {
  Grid<R> g(gg);
  R s = (R)0;
  for (int i = 0; i < N; ++i) {
    R x = (R)xyz[3 * i], y = (R)xyz[3 * i + 1], z = (R)xyz[3 * i + 2], gr[3] = {0, 0, 0};
    R v = interp == 0 ? nearest(g, x, y, z) : trilinear(g, x, y, z, gr);
    s = s + v;
    if (per_atom) per_atom[i] = (double)v;
    if (grad) for (int a = 0; a < 3; ++a) grad[3 * i + a] = (double)gr[a];
  }
  return (double)s;
}

extern "C" double oracle_score(int real_bits, const og_grid* g, int interp, int N, const double* xyz,
                    double* per_atom, double* grad) {
  return real_bits == 32 ? score_t<float>(g, interp, N, xyz, per_atom, grad)
                         : score_t<double>(g, interp, N, xyz, per_atom, grad);
}

// Trilinear score of a pose and its gradient with respect to the local
// parameters (t[3], omega[3], theta[K]) at zero (force / torque form):
//   dS/dt = sum_a g_a;  dS/domega = sum_a (x_a - P) x g_a;
//   dS/dtheta_k = u_k . sum_{a in F_k} (x_a - x_{a_k}) x g_a,  u_k = unit bond axis.
// g_a is the trilinear gradient at atom a.  FP64 only.
extern "C" double oracle_pose_grad(const og_grid* gg, const og_ligand* l, const double* xyz, const double* P,
                        double* grad) {
  Grid<double> g(gg);
  int N = l->N, K = l->K;
  std::vector<double> ga((size_t)3 * N);
  double s = 0;
  for (int i = 0; i < N; ++i) s += trilinear(g, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], &ga[3 * i]);
  for (int q = 0; q < 6 + K; ++q) grad[q] = 0;
  for (int i = 0; i < N; ++i) {
    const double* x = &xyz[3 * i];
    const double* gi = &ga[3 * i];
    double r[3] = {x[0] - P[0], x[1] - P[1], x[2] - P[2]};
    grad[0] += gi[0]; grad[1] += gi[1]; grad[2] += gi[2];
    grad[3] += r[1] * gi[2] - r[2] * gi[1];
    grad[4] += r[2] * gi[0] - r[0] * gi[2];
    grad[5] += r[0] * gi[1] - r[1] * gi[0];
  }
  for (int k = 0; k < K; ++k) {
    int a = l->ta[k], b = l->tb[k];
    double u[3] = {xyz[3 * b] - xyz[3 * a], xyz[3 * b + 1] - xyz[3 * a + 1], xyz[3 * b + 2] - xyz[3 * a + 2]};
    double nu = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) u[d] /= nu;
    double tq[3] = {0, 0, 0};
    for (int i = 0; i < N; ++i) {
      if (!((l->mask[i] >> k) & 1u)) continue;
      double r[3] = {xyz[3 * i] - xyz[3 * a], xyz[3 * i + 1] - xyz[3 * a + 1], xyz[3 * i + 2] - xyz[3 * a + 2]};
      const double* gi = &ga[3 * i];
      tq[0] += r[1] * gi[2] - r[2] * gi[1];
      tq[1] += r[2] * gi[0] - r[0] * gi[2];
      tq[2] += r[0] * gi[1] - r[1] * gi[0];
    }
    grad[6 + k] = u[0] * tq[0] + u[1] * tq[1] + u[2] * tq[2];
  }
  return s;
}

// Pose map of the local parameters q = (t[3], omega[3], theta[K]) applied to a
// pose (xyz, pivot P): torsions in reverse bond order about the current bond axes,
// then Exp(omega) about P, then + t.  FP64.
extern "C" int oracle_pose_map(const og_ligand* l, const double* xyz, const double* P, const double* q, double* out) {
  int N = l->N, K = l->K;
  std::vector<double> x(xyz, xyz + 3 * N);
  for (int k = K - 1; k >= 0; --k) {
    if (q[6 + k] == 0.0) continue;
    int a = l->ta[k], b = l->tb[k];
    double u[3] = {x[3 * b] - x[3 * a], x[3 * b + 1] - x[3 * a + 1], x[3 * b + 2] - x[3 * a + 2]};
    double nu = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) u[d] /= nu;
    double m[9];
    rodrigues(u, q[6 + k], m);
    for (int i = 0; i < N; ++i) {
      if (!((l->mask[i] >> k) & 1u) || i == b) continue;
      double v[3] = {x[3 * i] - x[3 * a], x[3 * i + 1] - x[3 * a + 1], x[3 * i + 2] - x[3 * a + 2]};
      for (int d = 0; d < 3; ++d) x[3 * i + d] = x[3 * a + d] + m[3 * d] * v[0] + m[3 * d + 1] * v[1] + m[3 * d + 2] * v[2];
    }
  }
  double w = std::sqrt(q[3] * q[3] + q[4] * q[4] + q[5] * q[5]);
  if (w > 0) {
    double u[3] = {q[3] / w, q[4] / w, q[5] / w}, m[9];
    rodrigues(u, w, m);
    for (int i = 0; i < N; ++i) {
      double v[3] = {x[3 * i] - P[0], x[3 * i + 1] - P[1], x[3 * i + 2] - P[2]};
      for (int d = 0; d < 3; ++d) x[3 * i + d] = P[d] + m[3 * d] * v[0] + m[3 * d + 1] * v[1] + m[3 * d + 2] * v[2];
    }
  }
  for (int i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) out[3 * i + d] = x[3 * i + d] + q[d];
  return 0;
}

// Top-k of R scores: order by score descending, equal scores by lower index.
extern "C" int oracle_topk(int R, const double* scores, int k, int32_t* out_idx) {
  std::vector<int> idx(R);
  for (int i = 0; i < R; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (scores[a] != scores[b]) return scores[a] > scores[b];
    return a < b;
  });
  for (int i = 0; i < k && i < R; ++i) out_idx[i] = idx[i];
  return 0;
}


// Local refinement of one pose (xyz, pivot P).  prm = (steps, eta_t, eta_w,
// eta_th, clip_t, clip_w, clip_th, clash2).  Returns the best score; out_xyz
// receives the best pose; *accepted the number of accepted steps.
extern "C" double oracle_refine(int real_bits, const og_grid* g, const og_ligand* l, const double* P,
                                const double* prm, double* out_xyz, int* accepted) {
  return real_bits == 32 ? refine_t<float>(g, l, P, prm, out_xyz, accepted)
                         : refine_t<double>(g, l, P, prm, out_xyz, accepted);
}

// The local move q = (t, omega, theta) applied to a pose (as refinement applies it).
extern "C" int oracle_apply_move(int real_bits, const og_ligand* l, const double* xyz, const double* P,
                                 const double* q, double* out_xyz, double* out_P) {
  return real_bits == 32 ? apply_move_t<float>(l, xyz, P, q, out_xyz, out_P)
                         : apply_move_t<double>(l, xyz, P, q, out_xyz, out_P);
}

// Trilinear score and gradient with respect to the local move at zero, as
// refinement computes it (axes from inv_len, sums in atom order).
extern "C" double oracle_move_grad(int real_bits, const og_grid* g, const og_ligand* l, const double* xyz,
                                   const double* P, double* grad) {
  return real_bits == 32 ? move_grad_t<float>(g, l, xyz, P, grad) : move_grad_t<double>(g, l, xyz, P, grad);
}

// 1 if the pose satisfies refinement's clash rule.
extern "C" int oracle_move_clash_free(int real_bits, const og_ligand* l, const double* xyz, double clash2) {
  return real_bits == 32 ? move_clash_free_t<float>(l, xyz, clash2) : move_clash_free_t<double>(l, xyz, clash2);
}
