// Seeded synthetic-input generators for the docking hot path.
//
// This module only *builds inputs*: a protein-pocket grid, ligand trees with
// their rotatable bonds, the restart table and the angle table.  It holds none
// of the docking method's arithmetic (no scans, no scoring, no clash rule), and
// both the GPU library and the CPU oracle consume what it writes.
//
// Every random draw comes from a counter-based SplitMix64 stream keyed by
// (seed, stream id, item id), so ligand i is the same whatever batch it sits
// in.  Stream ids: 1 pocket, 2 ligand sizes, 21 ligand geometry, 3 restarts,
// 4 sampled poses, 5 oracle subsets.
//
// The recipe follows the paper's workload framing: ligands whose cost depends
// on their atom and rotamer counts (Sec. 3), docked in a pocket grid.  The
// grid recipe (Gaussian attraction, shell repulsion, 2^-10 quantisation) and
// tree recipe are this project's stand-ins for the paper's unpublished data.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

inline uint64_t sm64_mix(uint64_t z) {
  // SplitMix64 finaliser (Steele, Lea, Flood 2014).
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct Rng {
  uint64_t s;
  Rng(uint64_t seed, uint64_t stream, uint64_t item) {
    const uint64_t g = 0x9E3779B97F4A7C15ULL;
    s = sm64_mix(sm64_mix(sm64_mix(seed + g) + stream * g) + item * g + 1);
  }
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ULL;
    return sm64_mix(s);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }       // [0,1)
  double uniform(double a, double b) { return a + (b - a) * uniform(); }
  int64_t integer(int64_t lo, int64_t hi) {                               // [lo,hi]
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)(next() % span);
  }
  double normal() {                                                       // Box-Muller
    double u1 = uniform(), u2 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  }
};

struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) { return (1.0 / norm(a)) * a; }

V3 uniform_sphere(Rng& r) {
  double z = 2.0 * r.uniform() - 1.0, p = 2.0 * M_PI * r.uniform();
  double s = std::sqrt(std::max(0.0, 1.0 - z * z));
  return {s * std::cos(p), s * std::sin(p), z};
}

V3 uniform_ball(Rng& r, double radius) {
  for (;;) {
    V3 v{r.uniform(-1, 1), r.uniform(-1, 1), r.uniform(-1, 1)};
    if (dot(v, v) <= 1.0) return radius * v;
  }
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------- pocket grid
// Node-centred grid of n^3 float32 values, x fastest: value(ix,iy,iz) sits at
// origin + (ix,iy,iz)*h and origin = center - (n-1)h/2.  Value = sum of n_gauss
// Gaussians (centres uniform in a 6 A ball about the centre, amplitude U[0.2,1],
// sigma 1.5 A), minus 5 once for every node within 2 A of any of n_shell shell
// atoms (radius U[6,8] A, direction uniform outside a 45-degree cone about +z,
// which stays open as the pocket mouth).  Values are rounded to a multiple of
// 2^-10 (nearest-even in FP64) and clamped to [-63, 63]; every sum of up to 256
// such values is then exact in FP32.  Returns 0 on success.
int gen_pocket(int n, double h, int n_gauss, int n_shell, uint64_t seed,
               const double* center, float* grid_out, float* origin_out) {
  if (n <= 1 || h <= 0) return -1;
  Rng rng(seed, 1, 0);
  const double sigma = 1.5, inv2s2 = 1.0 / (2.0 * sigma * sigma);
  V3 c{center[0], center[1], center[2]};
  V3 o = c - (0.5 * (n - 1) * h) * V3{1, 1, 1};
  std::vector<double> val((size_t)n * n * n, 0.0);
  std::vector<double> ex(n), ey(n), ez(n);
  for (int g = 0; g < n_gauss; ++g) {
    V3 gc = c + uniform_ball(rng, 6.0);
    double amp = rng.uniform(0.2, 1.0);
    for (int i = 0; i < n; ++i) {
      double px = o.x + i * h - gc.x, py = o.y + i * h - gc.y, pz = o.z + i * h - gc.z;
      ex[i] = std::exp(-px * px * inv2s2);
      ey[i] = std::exp(-py * py * inv2s2);
      ez[i] = amp * std::exp(-pz * pz * inv2s2);
    }
    for (int iz = 0; iz < n; ++iz)
      for (int iy = 0; iy < n; ++iy) {
        double zy = ez[iz] * ey[iy];
        double* row = &val[((size_t)iz * n + iy) * n];
        for (int ix = 0; ix < n; ++ix) row[ix] += zy * ex[ix];
      }
  }
  std::vector<uint8_t> near((size_t)n * n * n, 0);
  const double cone = std::cos(45.0 * M_PI / 180.0);
  for (int a = 0; a < n_shell; ++a) {
    V3 d;
    do { d = uniform_sphere(rng); } while (d.z > cone);
    V3 p = c + rng.uniform(6.0, 8.0) * d;
    int lo[3], hi[3];
    double pc[3] = {p.x, p.y, p.z}, oc[3] = {o.x, o.y, o.z};
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::max(0, (int)std::floor((pc[k] - 2.0 - oc[k]) / h));
      hi[k] = std::min(n - 1, (int)std::ceil((pc[k] + 2.0 - oc[k]) / h));
    }
    for (int iz = lo[2]; iz <= hi[2]; ++iz)
      for (int iy = lo[1]; iy <= hi[1]; ++iy)
        for (int ix = lo[0]; ix <= hi[0]; ++ix) {
          V3 q{o.x + ix * h, o.y + iy * h, o.z + iz * h};
          V3 dd = q - p;
          if (dot(dd, dd) <= 4.0) near[((size_t)iz * n + iy) * n + ix] = 1;
        }
  }
  for (size_t i = 0; i < val.size(); ++i) {
    double v = val[i] - (near[i] ? 5.0 : 0.0);
    v = std::nearbyint(v * 1024.0) / 1024.0;
    v = std::min(63.0, std::max(-63.0, v));
    grid_out[i] = (float)v;
  }
  origin_out[0] = (float)o.x; origin_out[1] = (float)o.y; origin_out[2] = (float)o.z;
  return 0;
}

// ------------------------------------------------------------ ligand sizes
// mode 0: N ~ U[nlo,nhi], K ~ U[klo,khi] (integers, inclusive).
// mode 1: lognormal atoms, N = clip(round(median*exp(0.4 z)), nlo, nhi) and
//         K = clip(round_half_even(0.18 N + 2 z'), klo, khi).
// Sizes of ligand ids[i] come from stream (seed, 2, ids[i]).
int gen_ligand_sizes(int count, const int64_t* ids, uint64_t seed, int mode,
                     int nlo, int nhi, int klo, int khi, double median,
                     int32_t* n_out, int32_t* k_out) {
  for (int i = 0; i < count; ++i) {
    Rng r(seed, 2, (uint64_t)ids[i]);
    int N, K;
    if (mode == 0) {
      N = (int)r.integer(nlo, nhi);
      K = (int)r.integer(klo, khi);
    } else {
      double z = r.normal(), z2 = r.normal();
      double nf = std::nearbyint(median * std::exp(0.4 * z));
      N = (int)std::min<double>(nhi, std::max<double>(nlo, nf));
      double kf = std::nearbyint(0.18 * N + 2.0 * z2);
      K = (int)std::min<double>(khi, std::max<double>(klo, kf));
    }
    n_out[i] = N; k_out[i] = K;
  }
  return 0;
}

// ------------------------------------------------------------ ligand geometry
// Builds one random tree ligand of N atoms (1.5 A bonds, 109.47 degree angle to
// the reference bond at the parent, uniform dihedral, every bond at a parent at
// least 100 degrees from the others, atoms 3+ bonds apart at least 2.4 A apart),
// renumbers it in DFS preorder (so every subtree is a contiguous index range),
// and picks up to K rotatable bonds among bonds whose two ends both have degree
// >= 2.  Bond k is (a_k, b_k) = (parent, child); its moving fragment is the
// subtree of b_k, recorded as bit k of frag_mask.  Bonds are ordered by b_k.
// Outputs (capacity N for atoms, K for bonds): xyz (FP64, atom-major 3N),
// parent (preorder ids, -1 for the root), tors_a/tors_b, frag_mask.  Returns the
// realised number of rotatable bonds, or -1 if the tree could not be grown.
static int build_one(int N, int K, Rng& r, double* xyz, int32_t* parent_out,
                     int32_t* ta, int32_t* tb, uint32_t* mask) {
  std::vector<V3> pos(N);
  std::vector<int> par(N, -1), deg(N, 0);
  std::vector<std::vector<int>> kids(N);
  std::vector<int> topo((size_t)N * N, 0);
  pos[0] = {0, 0, 0};
  const double cos_t = -1.0 / 3.0, sin_t = std::sqrt(8.0 / 9.0);
  const double min_cos_other = std::cos(100.0 * M_PI / 180.0);
  for (int a = 1; a < N; ++a) {
    bool placed = false;
    for (int pt = 0; pt < 4000 && !placed; ++pt) {
      std::vector<int> open;
      for (int i = 0; i < a; ++i) if (deg[i] < 4) open.push_back(i);
      if (open.empty()) return -1;
      int p = open[(size_t)r.integer(0, (int64_t)open.size() - 1)];
      int ref = par[p] >= 0 ? par[p] : (kids[p].empty() ? -1 : kids[p][0]);
      for (int tries = 0; tries < 100 && !placed; ++tries) {
        V3 d;
        if (ref < 0) {
          d = uniform_sphere(r);
        } else {
          V3 e = unit(pos[ref] - pos[p]);
          V3 helper = std::fabs(e.x) > 0.9 ? V3{0, 1, 0} : V3{1, 0, 0};
          V3 u1 = unit(cross(e, helper)), u2 = cross(e, u1);
          double phi = 2.0 * M_PI * r.uniform();
          d = cos_t * e + sin_t * (std::cos(phi) * u1 + std::sin(phi) * u2);
        }
        V3 cand = pos[p] + 1.5 * d;
        bool ok = true;
        std::vector<int> nb = kids[p];
        if (par[p] >= 0) nb.push_back(par[p]);
        for (int q : nb)
          if (dot(unit(pos[q] - pos[p]), d) > min_cos_other + 1e-12) { ok = false; break; }
        for (int i = 0; ok && i < a; ++i) {
          int t = topo[(size_t)p * N + i] + 1;
          if (t >= 3) {
            V3 dd = cand - pos[i];
            if (dot(dd, dd) < 2.4 * 2.4) ok = false;
          }
        }
        if (!ok) continue;
        pos[a] = cand; par[a] = p; deg[a] = 1; deg[p] += 1; kids[p].push_back(a);
        for (int i = 0; i < a; ++i) {
          topo[(size_t)a * N + i] = topo[(size_t)p * N + i] + 1;
          topo[(size_t)i * N + a] = topo[(size_t)a * N + i];
        }
        placed = true;
      }
    }
    if (!placed) return -1;
  }
  // DFS preorder renumbering, children in attachment order.
  std::vector<int> order, stack{0}, newid(N);
  while (!stack.empty()) {
    int v = stack.back(); stack.pop_back();
    order.push_back(v);
    for (auto it = kids[v].rbegin(); it != kids[v].rend(); ++it) stack.push_back(*it);
  }
  for (int i = 0; i < N; ++i) newid[order[i]] = i;
  std::vector<int> npar(N), ndeg(N), size(N, 1);
  for (int i = 0; i < N; ++i) {
    int v = order[i];
    xyz[3 * i] = pos[v].x; xyz[3 * i + 1] = pos[v].y; xyz[3 * i + 2] = pos[v].z;
    npar[i] = par[v] < 0 ? -1 : newid[par[v]];
    ndeg[i] = deg[v];
    parent_out[i] = npar[i];
  }
  for (int i = N - 1; i > 0; --i) size[npar[i]] += size[i];
  // Rotatable-bond candidates, listed by child (moving-side) preorder id.
  std::vector<int> cand;
  for (int i = 1; i < N; ++i)
    if (ndeg[i] >= 2 && ndeg[npar[i]] >= 2) cand.push_back(i);
  int Kr = std::min<int>(K, (int)cand.size());
  for (int i = 0; i < Kr; ++i) {                       // partial Fisher-Yates
    int j = (int)r.integer(i, (int64_t)cand.size() - 1);
    std::swap(cand[i], cand[j]);
  }
  std::vector<int> chosen(cand.begin(), cand.begin() + Kr);
  std::sort(chosen.begin(), chosen.end());
  for (int i = 0; i < N; ++i) mask[i] = 0;
  for (int k = 0; k < Kr; ++k) {
    int b = chosen[k];
    ta[k] = npar[b]; tb[k] = b;
    for (int i = b; i < b + size[b]; ++i) mask[i] |= (1u << k);
  }
  return Kr;
}

// Builds ligands ids[0..count) with sizes n_in/k_in (from gen_ligand_sizes).
// CSR outputs: atom arrays are indexed by atom_offset (prefix of n_in), bond
// arrays by bond_offset (prefix of k_in, i.e. the requested capacity).  The
// realised K of each ligand goes to k_out (<= k_in).  Per-ligand outputs:
// xyz64 (3 per atom, FP64), parent, frag_mask, tors_a/tors_b (local ids).
// Geometry of ligand ids[i] comes from stream (seed, 21, ids[i]).
int gen_ligands(int count, const int64_t* ids, uint64_t seed,
                const int32_t* n_in, const int32_t* k_in,
                const int64_t* atom_offset, const int64_t* bond_offset,
                double* xyz64, int32_t* parent, uint32_t* frag_mask,
                int32_t* tors_a, int32_t* tors_b, int32_t* k_out) {
  for (int i = 0; i < count; ++i) {
    if (n_in[i] < 1 || n_in[i] > 256 || k_in[i] < 0 || k_in[i] > 32) return -2;
    Rng r(seed, 21, (uint64_t)ids[i]);
    int64_t ao = atom_offset[i], bo = bond_offset[i];
    int kr = build_one(n_in[i], k_in[i], r, xyz64 + 3 * ao, parent + ao,
                       tors_a + bo, tors_b + bo, frag_mask + ao);
    if (kr < 0) return -1;
    k_out[i] = kr;
  }
  return 0;
}

// ---------------------------------------------------------------- restarts
// Row r (12 values): row-major 3x3 rotation, then an offset.  Row 0 is the
// identity with zero offset; other rows are a uniform rotation (Shoemake's
// quaternion method) and an offset uniform in a ball of radius `radius`.
// Written in FP64 (out64) and rounded to FP32 (out32).  Stream (seed, 3, r).
int gen_restarts(int R, uint64_t seed, double radius, double* out64, float* out32) {
  for (int r = 0; r < R; ++r) {
    double m[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
    if (r > 0) {
      Rng g(seed, 3, (uint64_t)r);
      double u1 = g.uniform(), u2 = g.uniform(), u3 = g.uniform();
      double a = std::sqrt(1 - u1), b = std::sqrt(u1);
      double qx = a * std::sin(2 * M_PI * u2), qy = a * std::cos(2 * M_PI * u2);
      double qz = b * std::sin(2 * M_PI * u3), qw = b * std::cos(2 * M_PI * u3);
      m[0] = 1 - 2 * (qy * qy + qz * qz); m[1] = 2 * (qx * qy - qz * qw); m[2] = 2 * (qx * qz + qy * qw);
      m[3] = 2 * (qx * qy + qz * qw); m[4] = 1 - 2 * (qx * qx + qz * qz); m[5] = 2 * (qy * qz - qx * qw);
      m[6] = 2 * (qx * qz - qy * qw); m[7] = 2 * (qy * qz + qx * qw); m[8] = 1 - 2 * (qx * qx + qy * qy);
      V3 t = uniform_ball(g, radius);
      m[9] = t.x; m[10] = t.y; m[11] = t.z;
    }
    for (int k = 0; k < 12; ++k) { out64[12 * r + k] = m[k]; out32[12 * r + k] = (float)m[k]; }
  }
  return 0;
}

// ------------------------------------------------------------- angle table
// Sample j of A is the angle 2*pi*j/A: (cos, sin) in FP64 and rounded to FP32,
// with exact 0 / +-1 at quarter turns.
int gen_angles(int A, double* out64, float* out32) {
  for (int j = 0; j < A; ++j) {
    double c, s;
    if ((4LL * j) % A == 0) {
      int q = (int)((4LL * j) / A);
      const double cq[4] = {1, 0, -1, 0}, sq[4] = {0, 1, 0, -1};
      c = cq[q]; s = sq[q];
    } else {
      double th = 2.0 * M_PI * (double)j / (double)A;
      c = std::cos(th); s = std::sin(th);
    }
    out64[2 * j] = c; out64[2 * j + 1] = s;
    out32[2 * j] = (float)c; out32[2 * j + 1] = (float)s;
  }
  return 0;
}

// ------------------------------------------------------ sampled parameters
// count x dim values uniform in [-scale, scale], stream (seed, stream, item).
int gen_uniform(int64_t count, int dim, uint64_t seed, uint64_t stream, double scale, double* out) {
  for (int64_t i = 0; i < count; ++i) {
    Rng r(seed, stream, (uint64_t)i);
    for (int d = 0; d < dim; ++d) out[i * dim + d] = r.uniform(-scale, scale);
  }
  return 0;
}

}  // extern "C"
