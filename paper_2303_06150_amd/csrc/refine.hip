// Local refinement of poses on the trilinear grid (gradient ascent in the local
// parameters t, omega, theta) and the local move applied before scoring.
//
// One wavefront refines one pose; atom 64 s + lane sits in slot s.  Each step:
// trilinear values and gradients per atom, force / torque / per-bond torque
// sums in atom order (readlane), the clipped step, the local move (torsions
// in reverse bond order about the current bond axes, rotation about the pivot,
// translation), the intramolecular clash rule over every pair a torsion can
// move, accept (keep the best pose) or reject (halve the step scale).  The
// arithmetic is the CPU reference's FP32 script: sums in atom order, (cos, sin)
// of step angles from one fixed polynomial, correctly rounded sqrt and divide.
#include "lg_device.h"

namespace lg {

template <int NSLOT>
struct MoveState {
  float x[3][NSLOT];
  float piv[3];
};

// (cos, sin) of a move angle: the step polynomial inside refinement (angles
// clipped to pi/4), the library functions for arbitrary moves.
template <bool LIB>
__device__ __forceinline__ void move_cos_sin(float x, float& c, float& s) {
  if (LIB) {
    sincosf(x, &s, &c);
  } else {
    step_cos_sin(x, c, s);
  }
}

// Torsions in reverse bond order (k = K-1 .. 0; deepest first when bonds are
// listed parents first), each about the bond axis at that moment.  th holds
// the bond angles.
template <int NSLOT, bool LIB = false>
__device__ void apply_torsions(MoveState<NSLOT>& p, const uint32_t (&mk)[NSLOT], int N, int K, const int2* tors,
                               const float* inv_len, const float* th) {
  const int lane = lane_id();
  for (int k = K - 1; k >= 0; --k) {
    const float ang = th[k];
    if (ang == 0.f) continue;
    float c, s;
    move_cos_sin<LIB>(ang, c, s);
    const int a = tors[k].x, b = tors[k].y;
    const float xa = atom_value(p.x[0], a), ya = atom_value(p.x[1], a), za = atom_value(p.x[2], a);
    const float il = inv_len[k];
    const float ux = (atom_value(p.x[0], b) - xa) * il, uy = (atom_value(p.x[1], b) - ya) * il,
                uz = (atom_value(p.x[2], b) - za) * il;
    float m[9];
    torsion_matrix(ux, uy, uz, c, s, m);
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      const int at = sl * 64 + lane;
      if (at < N && ((mk[sl] >> k) & 1u) && at != b) {
        float y0, y1, y2;
        mat_apply(m, p.x[0][sl] - xa, p.x[1][sl] - ya, p.x[2][sl] - za, y0, y1, y2);
        p.x[0][sl] = xa + y0;
        p.x[1][sl] = ya + y1;
        p.x[2][sl] = za + y2;
      }
    }
  }
}

// Rotation by |w| about w/|w| through the pivot, then + t (pivot included).
// q holds t[3], w[3].
template <int NSLOT, bool LIB = false>
__device__ void apply_rigid(MoveState<NSLOT>& p, const float* q) {
  const float w2 = fmaf(q[5], q[5], fmaf(q[4], q[4], q[3] * q[3]));
  if (w2 > 0.f) {
    const float w = sqrtf(w2);
    float c, s, m[9];
    move_cos_sin<LIB>(w, c, s);
    torsion_matrix(q[3] / w, q[4] / w, q[5] / w, c, s, m);
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      float y0, y1, y2;
      mat_apply(m, p.x[0][sl] - p.piv[0], p.x[1][sl] - p.piv[1], p.x[2][sl] - p.piv[2], y0, y1, y2);
      p.x[0][sl] = p.piv[0] + y0;
      p.x[1][sl] = p.piv[1] + y1;
      p.x[2][sl] = p.piv[2] + y2;
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) p.x[d][sl] = p.x[d][sl] + q[d];
    p.piv[d] = p.piv[d] + q[d];
  }
}

// The same rigid move with the three divisions of the axis done by lanes 0..2
// at once (the same quotients; one division sequence instead of three).
template <int NSLOT>
__device__ void apply_rigid_lanes(MoveState<NSLOT>& p, const float* q) {
  const float w2 = fmaf(q[5], q[5], fmaf(q[4], q[4], q[3] * q[3]));
  if (w2 > 0.f) {
    const float w = sqrtf(w2);
    float c, s, m[9];
    step_cos_sin(w, c, s);
    const int lane = lane_id();
    const float num = lane == 0 ? q[3] : (lane == 1 ? q[4] : q[5]);
    const float u = num / w;
    const float ux = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 0));
    const float uy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 1));
    const float uz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 2));
    torsion_matrix(ux, uy, uz, c, s, m);
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      float y0, y1, y2;
      mat_apply(m, p.x[0][sl] - p.piv[0], p.x[1][sl] - p.piv[1], p.x[2][sl] - p.piv[2], y0, y1, y2);
      p.x[0][sl] = p.piv[0] + y0;
      p.x[1][sl] = p.piv[1] + y1;
      p.x[2][sl] = p.piv[2] + y2;
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) p.x[d][sl] = p.x[d][sl] + q[d];
    p.piv[d] = p.piv[d] + q[d];
  }
}

// The rigid move with its rotation matrix built beforehand (rows at M[0..2],
// as apply_torsions_table's); rot: the rotation angle is non-zero.
template <int NSLOT>
__device__ void apply_rigid_table(MoveState<NSLOT>& p, const float* q, bool rot, const float4* M) {
  if (rot) {
    const float4 r0 = M[0], r1 = M[1], r2 = M[2];
    const float m[9] = {r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, r2.x, r2.y, r2.z};
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      float y0, y1, y2;
      mat_apply(m, p.x[0][sl] - p.piv[0], p.x[1][sl] - p.piv[1], p.x[2][sl] - p.piv[2], y0, y1, y2);
      p.x[0][sl] = p.piv[0] + y0;
      p.x[1][sl] = p.piv[1] + y1;
      p.x[2][sl] = p.piv[2] + y2;
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) p.x[d][sl] = p.x[d][sl] + q[d];
    p.piv[d] = p.piv[d] + q[d];
  }
}

// The local move: torsions in reverse bond order, rotation about the pivot, translation.
template <int NSLOT, bool LIB = false>
__device__ void apply_move(MoveState<NSLOT>& p, const uint32_t (&mk)[NSLOT], int N, int K, const int2* tors,
                           const float* inv_len, const float* q, const float* th) {
  apply_torsions<NSLOT, LIB>(p, mk, N, K, tors, inv_len, th);
  apply_rigid<NSLOT, LIB>(p, q);
}

// Bond k's axis at the pose held in pos, computed by lane k: pivot atom a_k and
// unit direction (b_k - a_k) / |b_k - a_k| (the stored inverse length).
struct LaneAxis {
  float xa, ya, za, ux, uy, uz;
};

__device__ __forceinline__ LaneAxis lane_axis(const float4* pos, const int2* tors, const float* inv_len, int K) {
  LaneAxis ax{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int k = lane_id();
  if (k < K) {
    const int2 t = tors[k];
    const float4 pa = pos[t.x], pb = pos[t.y];
    const float il = inv_len[k];
    ax.xa = pa.x;
    ax.ya = pa.y;
    ax.za = pa.z;
    ax.ux = (pb.x - pa.x) * il;
    ax.uy = (pb.y - pa.y) * il;
    ax.uz = (pb.z - pa.z) * il;
  }
  return ax;
}

// Does a torsion ever move the axis atoms of a shallower bond?  When no bond j
// moves a_k or b_k of a bond k < j (bonds listed parents first, as a preorder
// numbering gives), every axis that the reverse-order sequence uses is the axis
// at the start of the move, so all torsion matrices can be built at once.
__device__ __forceinline__ bool axes_fixed_under_torsions(const LigDev& P, int abase, int toff, int K) {
  const int k = lane_id();
  bool moved = false;
  if (k < K && k + 1 < 32) {
    const int a = P.tors_atoms[2 * (toff + k)], b = P.tors_atoms[2 * (toff + k) + 1];
    moved = ((P.mask[abase + a] | P.mask[abase + b]) >> (k + 1)) != 0u;
  }
  return !wave_any(moved);
}

// Torsions in reverse bond order with matrices built beforehand: rows r of bond k at
// mats[3k + r] = (m[3r], m[3r+1], m[3r+2], pivot coordinate r).  Valid when the
// axes stay fixed under the torsions (axes_fixed_under_torsions).
// mv: per slot, the bonds that rotate the lane's atom (bit k of the fragment
// mask, cleared for b_k itself and for lanes past the last atom).
template <int NSLOT>
__device__ void apply_torsions_table(MoveState<NSLOT>& p, const uint32_t (&mv)[NSLOT], int K, const float* th,
                                     const float4* mats) {
  for (int k = K - 1; k >= 0; --k) {
    const float ang = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(th[k])));
    if (ang == 0.f) continue;
    const float4 r0 = mats[3 * k], r1 = mats[3 * k + 1], r2 = mats[3 * k + 2];
    const float m[9] = {r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, r2.x, r2.y, r2.z};
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      if ((mv[sl] >> k) & 1u) {
        float y0, y1, y2;
        mat_apply(m, p.x[0][sl] - r0.w, p.x[1][sl] - r1.w, p.x[2][sl] - r2.w, y0, y1, y2);
        p.x[0][sl] = r0.w + y0;
        p.x[1][sl] = r1.w + y1;
        p.x[2][sl] = r2.w + y2;
      }
    }
  }
}

// Per-atom columns summed in atom order through an LDS tile: the wavefront
// writes the columns of 64 atoms (one slot) as tile[column * TILE_STRIDE + lane],
// then lane c adds column c's values atom by atom, four per LDS read.  Each
// column's sum runs over atoms 0..N-1 in order, like a sequential loop, but all
// columns at once.
constexpr int TILE_COLS = 16;                      // LDS per wavefront stays small (occupancy)
constexpr int TILE_STRIDE = 68;                    // 16-byte aligned columns for 4-float reads
constexpr int TILE_FLOATS = TILE_COLS * TILE_STRIDE;
constexpr int GRAD_COLS = 7 + 3 * 32;              // score, force, torque, 3 per bond
constexpr int GRAD_RES_FLOATS = 104;               // GRAD_COLS rounded up to float4
constexpr int GRAD_LDS_FLOAT4 = (TILE_FLOATS + GRAD_RES_FLOATS) / 4;
static_assert(GRAD_RES_FLOATS >= GRAD_COLS && GRAD_RES_FLOATS % 4 == 0, "gradient results: every column, whole float4");
static_assert(TILE_FLOATS >= 12 * 32, "the torsion matrices reuse the tile");

// Trilinear score and its gradient with respect to the local move at zero;
// sums in atom order.  g_out: t[3], w[3], then theta[K] into th_grad.  Column
// 0 is the score, 1..3 the force, 4..6 the torque about the pivot, 7 + 3k + d
// component d of bond k's torque about its pivot atom over F_k.  pos holds the
// pose p; lane k holds bond k's axis.
template <int NSLOT>
__device__ float move_gradient(const GridDev& G, const MoveState<NSLOT>& p, const uint32_t (&mk)[NSLOT], int N,
                               int K, const int2* tors, const float4* pos, const LaneAxis& ax, float* g_out,
                               float* th_grad, float* tile, float* res) {
  const int lane = lane_id();
  float v[NSLOT], g[3][NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    float gg[3] = {0.f, 0.f, 0.f};
    v[s] = (s * 64 + lane < N) ? trilinear(G, p.x[0][s], p.x[1][s], p.x[2][s], gg) : 0.f;
    g[0][s] = gg[0]; g[1][s] = gg[1]; g[2][s] = gg[2];
  }
  // column chunks: the 7 pose columns with bonds 0..2, then 5 bonds per chunk
  for (int k0 = 0, first = 1; first || k0 < K; first = 0) {
    const int base = first ? 7 : 0;
    const int nb = min(K - k0, (TILE_COLS - base) / 3);
    const int ncol = base + 3 * nb;
    const int col0 = first ? 0 : 7 + 3 * k0;
    float acc = 0.f;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int cnt = min(64, N - s * 64);
      if (cnt <= 0) break;
      if (first) {
        const float r0 = p.x[0][s] - p.piv[0], r1 = p.x[1][s] - p.piv[1], r2 = p.x[2][s] - p.piv[2];
        tile[0 * TILE_STRIDE + lane] = v[s];
        tile[1 * TILE_STRIDE + lane] = g[0][s];
        tile[2 * TILE_STRIDE + lane] = g[1][s];
        tile[3 * TILE_STRIDE + lane] = g[2][s];
        tile[4 * TILE_STRIDE + lane] = r1 * g[2][s] - r2 * g[1][s];
        tile[5 * TILE_STRIDE + lane] = r2 * g[0][s] - r0 * g[2][s];
        tile[6 * TILE_STRIDE + lane] = r0 * g[1][s] - r1 * g[0][s];
      }
      for (int kk = 0; kk < nb; ++kk) {
        const int k = k0 + kk;
        const float4 pa = pos[tors[k].x];   // pivot atom a_k, the same address in every lane
        const bool in = (mk[s] >> k) & 1u;
        const float r0 = p.x[0][s] - pa.x, r1 = p.x[1][s] - pa.y, r2 = p.x[2][s] - pa.z;
        float* t = tile + (base + 3 * kk) * TILE_STRIDE + lane;
        t[0] = in ? r1 * g[2][s] - r2 * g[1][s] : 0.f;
        t[TILE_STRIDE] = in ? r2 * g[0][s] - r0 * g[2][s] : 0.f;
        t[2 * TILE_STRIDE] = in ? r0 * g[1][s] - r1 * g[0][s] : 0.f;
      }
      wave_sync();
      if (lane < ncol) {
        const float* col = tile + lane * TILE_STRIDE;
        int l = 0;
        for (; l + 4 <= cnt; l += 4) {
          const float4 q4 = *reinterpret_cast<const float4*>(col + l);
          acc = acc + q4.x;
          acc = acc + q4.y;
          acc = acc + q4.z;
          acc = acc + q4.w;
        }
        for (; l < cnt; ++l) acc = acc + col[l];
      }
      wave_sync();
    }
    if (lane < ncol) res[col0 + lane] = acc;
    k0 += nb;
  }
  wave_sync();
#pragma unroll
  for (int d = 0; d < 6; ++d) g_out[d] = res[1 + d];
  if (lane < K) {
    const float* t = res + 7 + 3 * lane;
    th_grad[lane] = ax.ux * t[0] + ax.uy * t[1] + ax.uz * t[2];
  }
  return res[0];
}

// Refinement clash rule: every pair that some bond's torsion moves -- exactly one
// of the two in F_k, the moving one not b_k, the other not a_k -- at squared
// distance >= clash2.  `pos` holds the pose (xyz, mask bits in w) in LDS,
// followed by a copy of its first (N - 1) / 2 atoms, so atom (i + d) mod N sits
// at pos[i + d].  Each unordered pair is visited once: the lane's atom i with
// atom i + d for d = 1 .. N/2 (for even N the pair at d = N/2 only from its
// lower end).  The distance test comes first; the bond rule is evaluated only
// when some lane holds a pair inside the clash distance (bonded neighbours),
// and the pass stops at the first clash, which already decides the step.
__device__ __forceinline__ bool pair_changes(uint32_t mi, uint32_t mj, int i, int j, const int2* tors) {
  bool changes = false;
  for (uint32_t m = mi ^ mj; m != 0u && !changes; m &= m - 1u) {
    const int k = __builtin_ctz(m);
    const int mover = ((mi >> k) & 1u) ? i : j;
    const int other = mover == i ? j : i;
    changes = mover != tors[k].y && other != tors[k].x;
  }
  return changes;
}

template <int NSLOT>
__device__ bool move_clash_free(const MoveState<NSLOT>& p, const uint32_t (&mk)[NSLOT], int N,
                                const int2* tors, const float4* pos, float clash2) {
  const int lane = lane_id();
  bool clash = false;
  const int half = N >> 1;
  const int full = (N - 1) >> 1;   // every d in 1 .. full from each atom; for even N also d = N/2 from the lower end
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    if (s * 64 >= N || wave_any(clash)) break;
    const int i = s * 64 + lane;
    if (i < N) {
      const float4* pi = pos + i;
      const float xi = p.x[0][s], yi = p.x[1][s], zi = p.x[2][s];
      auto near = [&](const float4& pj) {
        const float dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
        return fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < clash2;
      };
      auto rule = [&](int d, const float4& pj) {
        const int j = i + d >= N ? i + d - N : i + d;
        clash |= pair_changes(mk[s], __float_as_uint(pj.w), i, j, tors);
      };
      auto test = [&](int d) {
        const float4 pj = pi[d];
        const bool n0 = near(pj);
        if (__ballot(n0) != 0ull && n0) rule(d, pj);
      };
      int d = 1;
      for (; d + 3 <= full; d += 4) {   // four reads in flight, one vote for the rare bond rule
        const float4 p0 = pi[d], p1 = pi[d + 1], p2 = pi[d + 2], p3 = pi[d + 3];
        const bool n0 = near(p0), n1 = near(p1), n2 = near(p2), n3 = near(p3);
        if (__ballot(n0 || n1 || n2 || n3) != 0ull) {
          if (n0) rule(d, p0);
          if (n1) rule(d + 1, p1);
          if (n2) rule(d + 2, p2);
          if (n3) rule(d + 3, p3);
          if (__ballot(clash) != 0ull) break;   // one clash decides: the step is rejected
        }
      }
      if (__ballot(clash) == 0ull) {
        for (; d <= full; ++d) test(d);
        if (half > full && i < half) test(half);
      }
    }
  }
  return !wave_any(clash);
}

template <int NSLOT>
__device__ __forceinline__ void store_pose(float4* pos, const MoveState<NSLOT>& p, const uint32_t (&mk)[NSLOT],
                                           int N, bool wrap = false) {
  const int lane = lane_id();
  const int full = (N - 1) >> 1;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    const float4 v = make_float4(p.x[0][s], p.x[1][s], p.x[2][s], __uint_as_float(mk[s]));
    if (a < N) pos[a] = v;
    if (wrap && a < full) pos[N + a] = v;   // the copy the clash pass reads past atom N - 1
  }
}

// LDS of one refinement wavefront in float4: pose, gradient tile, bond atoms,
// 1/lengths, bond steps, bond gradients, gradient results.  The clash pass's
// copy of the first atoms runs from the pose into the tile's first 32 * nslot
// float4; the torsion matrices sit in the tile after it.
constexpr int refine_wave_float4(int nslot) { return 64 * nslot + 16 + 8 + 8 + 8 + GRAD_LDS_FLOAT4; }
constexpr int refine_mats_float4(int nslot) { return 32 * nslot; }
static_assert(refine_mats_float4(4) + 3 * 33 <= TILE_FLOATS / 4, "wrap copy and the matrices fit in the tile");

template <int NSLOT>
__global__ __launch_bounds__(256) void refine_kernel(GridDev G, LigDev P, RefineDev Rp, int n) {
  extern __shared__ float4 lds[];
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6, lane = lane_id();
  float4* pos = lds + (size_t)wave * refine_wave_float4(NSLOT);
  float* tile = reinterpret_cast<float*>(pos + 64 * NSLOT);   // column sums of the gradient; then wrap copy + matrices
  int2* tors = reinterpret_cast<int2*>(tile + TILE_FLOATS);   // 32 entries (16 float4)
  float* inv_len = reinterpret_cast<float*>(tors + 32);       // 32 entries (8 float4)
  float* th = inv_len + 32;                                   // 32 bond steps (8 float4)
  float* thg = th + 32;                                       // 32 bond gradients (8 float4)
  float* res = thg + 32;                                      // gradient results
  const int w = blockIdx.x * nwaves + wave;   // pose: member w % kpl of the launch's ligand w / kpl
  if (w >= n) return;
  const int li = w / Rp.kpl, member = w - li * Rp.kpl;
  const int lig = Rp.lig_ids ? __builtin_amdgcn_readfirstlane(Rp.lig_ids[li]) : li;
  const int i = lig * Rp.kpl + member;        // pose index in the caller's layout
  const int abase = __builtin_amdgcn_readfirstlane(P.atom_offset[lig]);
  const int N = __builtin_amdgcn_readfirstlane(P.atom_offset[lig + 1]) - abase;
  const int toff = __builtin_amdgcn_readfirstlane(P.tors_offset[lig]);
  const int K = __builtin_amdgcn_readfirstlane(P.tors_offset[lig + 1]) - toff;
  const size_t cbase = (size_t)Rp.kpl * abase + (size_t)member * N;   // coordinates of the pose
  if (lane < K) {
    tors[lane] = make_int2(P.tors_atoms[2 * (toff + lane)], P.tors_atoms[2 * (toff + lane) + 1]);
    inv_len[lane] = P.inv_len[toff + lane];
  }
  const bool table = axes_fixed_under_torsions(P, abase, toff, K);
  uint32_t mv[NSLOT];   // bonds that rotate the lane's atom (b_k excluded)
  MoveState<NSLOT> cur, best;
  uint32_t mk[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    const bool in = a < N;
    cur.x[0][s] = in ? P.x[cbase + a] : 0.f;
    cur.x[1][s] = in ? P.y[cbase + a] : 0.f;
    cur.x[2][s] = in ? P.z[cbase + a] : 0.f;
    mk[s] = in ? P.mask[abase + a] : 0u;
    mv[s] = mk[s];
  }
  for (int k = 0; k < K; ++k) {
    const int b = __builtin_amdgcn_readfirstlane(P.tors_atoms[2 * (toff + k) + 1]);
#pragma unroll
    for (int s = 0; s < NSLOT; ++s)
      if (s * 64 + lane == b) mv[s] &= ~(1u << k);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) cur.piv[d] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.ref[3 * i + d])));
  wave_sync();
  best = cur;
  float v[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) v[s] = (s * 64 + lane < N) ? trilinear(G, cur.x[0][s], cur.x[1][s], cur.x[2][s], nullptr) : 0.f;
  float best_s = atom_order_sum(v, N);
  float scale = 1.f;
  float g[6];
  LaneAxis ax;
  // fresh: cur changed since the last gradient (a rejected step keeps the pose,
  // so its gradient is reused); pending: cur was accepted and not yet compared
  // with the best -- the gradient pass's column 0 is its score
  bool fresh = true, pending = false;
  // pos holds cur whenever a gradient is due: here, and after an accepted step
  // (the candidate was stored for its clash pass)
  store_pose(pos, cur, mk, N);
  wave_sync();
  for (int step = 0; step < Rp.steps; ++step) {
    if (fresh) {
      ax = lane_axis(pos, tors, inv_len, K);
      const float sc = move_gradient(G, cur, mk, N, K, tors, pos, ax, g, thg, tile, res);
      wave_sync();
      if (pending && sc > best_s) {
        best_s = sc;
        best = cur;
      }
      fresh = pending = false;
    }
    float q[6];
    float dt[3], dw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) { dt[d] = Rp.eta_t * g[d]; dw[d] = Rp.eta_w * g[3 + d]; }
    // clip factors: lane 0 the translation's, lane 1 the rotation's
    float ft, fw;
    {
      const bool rot = lane == 1;
      const float a0 = rot ? dw[0] : dt[0], a1 = rot ? dw[1] : dt[1], a2 = rot ? dw[2] : dt[2];
      const float clip = rot ? Rp.clip_w : Rp.clip_t;
      const float nrm = sqrtf(fmaf(a2, a2, fmaf(a1, a1, a0 * a0)));
      const float f = nrm > clip ? clip / nrm : 1.f;
      ft = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), 0));
      fw = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), 1));
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      q[d] = (dt[d] * ft) * scale;
      q[3 + d] = (dw[d] * fw) * scale;
    }
    // bond k's step by lane k; with fixed axes also its matrix, into the tile
    float thk = 0.f;
    if (lane < K) {
      float t = Rp.eta_th * thg[lane];
      t = fminf(fmaxf(t, -Rp.clip_th), Rp.clip_th);
      thk = t * scale;
      th[lane] = thk;
    }
    MoveState<NSLOT> cand = cur;
    if (table) {
      // every matrix of the move in one pass: lane k < K bond k's, lane K the
      // rigid rotation's (axis w/|w| from three quotients by lanes 0..2)
      float4* mats = reinterpret_cast<float4*>(tile) + refine_mats_float4(NSLOT);
      const float w2 = fmaf(q[5], q[5], fmaf(q[4], q[4], q[3] * q[3]));
      const bool rot = w2 > 0.f;
      float wlen = 0.f, wx = 0.f, wy = 0.f, wz = 0.f;
      if (rot) {
        wlen = sqrtf(w2);
        const float num = lane == 0 ? q[3] : (lane == 1 ? q[4] : q[5]);
        const float u = num / wlen;
        wx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 0));
        wy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 1));
        wz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 2));
      }
      const bool bond = lane < K && thk != 0.f;
      if (bond || (lane == K && rot)) {
        const float ang = bond ? thk : wlen;
        const float ux = bond ? ax.ux : wx, uy = bond ? ax.uy : wy, uz = bond ? ax.uz : wz;
        float c, sn, m[9];
        step_cos_sin(ang, c, sn);
        torsion_matrix(ux, uy, uz, c, sn, m);
        mats[3 * lane] = make_float4(m[0], m[1], m[2], ax.xa);
        mats[3 * lane + 1] = make_float4(m[3], m[4], m[5], ax.ya);
        mats[3 * lane + 2] = make_float4(m[6], m[7], m[8], ax.za);
      }
      wave_sync();
      apply_torsions_table(cand, mv, K, th, mats);
      apply_rigid_table(cand, q, rot, mats + 3 * K);
    } else {
      wave_sync();
      apply_torsions(cand, mk, N, K, tors, inv_len, th);
      apply_rigid_lanes(cand, q);
    }
    store_pose(pos, cand, mk, N, true);
    wave_sync();
    const bool ok = move_clash_free(cand, mk, N, tors, pos, Rp.clash2);
    wave_sync();
    if (!ok) {
      scale = scale * 0.5f;
      continue;
    }
    cur = cand;
    fresh = pending = true;
  }
  if (pending) {   // the last step's accepted pose
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) v[s] = (s * 64 + lane < N) ? trilinear(G, cur.x[0][s], cur.x[1][s], cur.x[2][s], nullptr) : 0.f;
    const float sc = atom_order_sum(v, N);
    if (sc > best_s) {
      best_s = sc;
      best = cur;
    }
  }
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    if (a < N) {
      Rp.xo[cbase + a] = best.x[0][s];
      Rp.yo[cbase + a] = best.x[1][s];
      Rp.zo[cbase + a] = best.x[2][s];
    }
  }
  if (lane == 0) Rp.score[i] = best_s;
}

// ---- two poses per wavefront (ligands of at most 32 atoms) -------------------
// Poses 2m and 2m + 1 of one ligand share a wavefront: pose h = lane / 32 in
// lanes 32 h .. 32 h + 31, atom a in lane 32 h + a.  Both halves have the same
// atoms, bonds and fragment masks, so every loop bound and branch is the
// ligand's and the halves run one control flow; per-pose values (pivot, step,
// step scale, accept) are per lane.  Each half does exactly the arithmetic of
// refine_kernel<1> for its pose: the same sums in atom order, the same step
// script, the same clash rule.  A wavefront without a second pose (odd k)
// refines the first pose twice and stores it once.
constexpr int PAIR_STRIDE = 36;                              // 32 atoms + pad, 16-byte aligned columns
constexpr int PAIR_TILE_FLOATS = TILE_COLS * PAIR_STRIDE;    // per half
constexpr int PAIR_POS_FLOAT4 = 48;                          // 32 atoms + the clash pass's wrap copy
static_assert(PAIR_TILE_FLOATS / 4 >= 3 * 32, "the matrices of 31 bonds and the rigid move fit in a half's tile");
// LDS of one wavefront in float4: poses, tiles, bond atoms, 1/lengths, steps,
// bond gradients, gradient results
constexpr int pair_wave_float4() {
  return 2 * PAIR_POS_FLOAT4 + 2 * PAIR_TILE_FLOATS / 4 + 16 + 8 + 2 * 8 + 2 * 8 + 2 * GRAD_RES_FLOATS / 4;
}

__device__ __forceinline__ int half_of_lane() { return lane_id() >> 5; }

// Sum over atoms 0..N-1 of each half in atom order; every lane gets its half's.
__device__ __forceinline__ float pair_atom_order_sum(float v, int N) {
  float a = 0.f, b = 0.f;
  for (int l = 0; l < N; ++l) {
    a = a + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
    b = b + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32 + l));
  }
  return half_of_lane() ? b : a;
}

struct PairPose {
  float x[3];
  float piv[3];
};

// move_gradient for the two halves: columns per half in that half's tile, summed
// in atom order by lanes 32 h + c; results in that half's res.
__device__ float pair_move_gradient(const GridDev& G, const PairPose& p, uint32_t mk, int N, int K, const int2* tors,
                                    const float4* pos_h, const LaneAxis& ax, float (&g_out)[6], float* thg_h,
                                    float* tile_h, float* res_h) {
  const int la = lane_id() & 31;
  float gg[3] = {0.f, 0.f, 0.f};
  const float v = la < N ? trilinear(G, p.x[0], p.x[1], p.x[2], gg) : 0.f;
  for (int k0 = 0, first = 1; first || k0 < K; first = 0) {
    const int base = first ? 7 : 0;
    const int nb = min(K - k0, (TILE_COLS - base) / 3);
    const int ncol = base + 3 * nb;
    const int col0 = first ? 0 : 7 + 3 * k0;
    if (first) {
      const float r0 = p.x[0] - p.piv[0], r1 = p.x[1] - p.piv[1], r2 = p.x[2] - p.piv[2];
      tile_h[0 * PAIR_STRIDE + la] = v;
      tile_h[1 * PAIR_STRIDE + la] = gg[0];
      tile_h[2 * PAIR_STRIDE + la] = gg[1];
      tile_h[3 * PAIR_STRIDE + la] = gg[2];
      tile_h[4 * PAIR_STRIDE + la] = r1 * gg[2] - r2 * gg[1];
      tile_h[5 * PAIR_STRIDE + la] = r2 * gg[0] - r0 * gg[2];
      tile_h[6 * PAIR_STRIDE + la] = r0 * gg[1] - r1 * gg[0];
    }
    for (int kk = 0; kk < nb; ++kk) {
      const int k = k0 + kk;
      const float4 pa = pos_h[tors[k].x];   // pivot atom a_k of this half's pose
      const bool in = (mk >> k) & 1u;
      const float r0 = p.x[0] - pa.x, r1 = p.x[1] - pa.y, r2 = p.x[2] - pa.z;
      float* t = tile_h + (base + 3 * kk) * PAIR_STRIDE + la;
      t[0] = in ? r1 * gg[2] - r2 * gg[1] : 0.f;
      t[PAIR_STRIDE] = in ? r2 * gg[0] - r0 * gg[2] : 0.f;
      t[2 * PAIR_STRIDE] = in ? r0 * gg[1] - r1 * gg[0] : 0.f;
    }
    wave_sync();
    float acc = 0.f;
    if (la < ncol) {
      const float* col = tile_h + la * PAIR_STRIDE;
      int l = 0;
      for (; l + 4 <= N; l += 4) {
        const float4 q4 = *reinterpret_cast<const float4*>(col + l);
        acc = acc + q4.x;
        acc = acc + q4.y;
        acc = acc + q4.z;
        acc = acc + q4.w;
      }
      for (; l < N; ++l) acc = acc + col[l];
    }
    wave_sync();
    if (la < ncol) res_h[col0 + la] = acc;
    k0 += nb;
  }
  wave_sync();
#pragma unroll
  for (int d = 0; d < 6; ++d) g_out[d] = res_h[1 + d];
  if (la < K) {
    const float* t = res_h + 7 + 3 * la;
    thg_h[la] = ax.ux * t[0] + ax.uy * t[1] + ax.uz * t[2];
  }
  return res_h[0];
}

// Clash rule of refinement for both halves (as move_clash_free, atom i of each
// half against atoms i + d of its own pose): the result of the lane's half.  The
// pass stops once both halves have found a clash.
__device__ bool pair_clash_free(const PairPose& p, uint32_t mk, int N, const int2* tors, const float4* pos_h,
                                float clash2) {
  const int la = lane_id() & 31;
  const uint64_t lo_half = 0x00000000FFFFFFFFull, hi_half = ~lo_half;
  auto both = [&](uint64_t b) { return (b & lo_half) != 0ull && (b & hi_half) != 0ull; };
  bool clash = false;
  const int half = N >> 1;
  const int full = (N - 1) >> 1;
  if (la < N) {
    const float4* pi = pos_h + la;
    const float xi = p.x[0], yi = p.x[1], zi = p.x[2];
    auto near = [&](const float4& pj) {
      const float dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
      return fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < clash2;
    };
    auto rule = [&](int d, const float4& pj) {
      const int j = la + d >= N ? la + d - N : la + d;
      clash |= pair_changes(mk, __float_as_uint(pj.w), la, j, tors);
    };
    auto test = [&](int d) {
      const float4 pj = pi[d];
      const bool n0 = near(pj);
      if (__ballot(n0) != 0ull && n0) rule(d, pj);
    };
    int d = 1;
    for (; d + 3 <= full; d += 4) {
      const float4 p0 = pi[d], p1 = pi[d + 1], p2 = pi[d + 2], p3 = pi[d + 3];
      const bool n0 = near(p0), n1 = near(p1), n2 = near(p2), n3 = near(p3);
      if (__ballot(n0 || n1 || n2 || n3) != 0ull) {
        if (n0) rule(d, p0);
        if (n1) rule(d + 1, p1);
        if (n2) rule(d + 2, p2);
        if (n3) rule(d + 3, p3);
        if (both(__ballot(clash))) break;
      }
    }
    if (!both(__ballot(clash))) {
      for (; d <= full; ++d) test(d);
      if (half > full && la < half) test(half);
    }
  }
  const uint64_t b = __ballot(clash);
  return (b & (half_of_lane() ? hi_half : lo_half)) == 0ull;
}

__device__ __forceinline__ void pair_store_pose(float4* pos_h, const PairPose& p, uint32_t mk, int N, bool wrap) {
  const int la = lane_id() & 31;
  const int full = (N - 1) >> 1;
  const float4 v = make_float4(p.x[0], p.x[1], p.x[2], __uint_as_float(mk));
  if (la < N) pos_h[la] = v;
  if (wrap && la < full) pos_h[N + la] = v;
}

__global__ __launch_bounds__(256) void refine_pair_kernel(GridDev G, LigDev P, RefineDev Rp, int n_pairs) {
  extern __shared__ float4 lds[];
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6, lane = lane_id();
  const int h = lane >> 5, la = lane & 31;
  float4* base4 = lds + (size_t)wave * pair_wave_float4();
  float4* pos_h = base4 + h * PAIR_POS_FLOAT4;
  float* tile_h = reinterpret_cast<float*>(base4 + 2 * PAIR_POS_FLOAT4) + h * PAIR_TILE_FLOATS;
  int2* tors = reinterpret_cast<int2*>(base4 + 2 * PAIR_POS_FLOAT4 + 2 * PAIR_TILE_FLOATS / 4);   // 32 entries
  float* inv_len = reinterpret_cast<float*>(tors + 32);                                          // 32 entries
  float* th_h = inv_len + 32 + h * 32;        // bond steps of this half's pose
  float* thg_h = inv_len + 96 + h * 32;       // bond gradients
  float* res_h = inv_len + 160 + h * GRAD_RES_FLOATS;
  const int w = blockIdx.x * nwaves + wave;   // pair w: members 2m, 2m + 1 of ligand w / ppl
  if (w >= n_pairs) return;
  const int ppl = (Rp.kpl + 1) >> 1;
  const int li = w / ppl, m = w - li * ppl;
  const int lig = Rp.lig_ids ? __builtin_amdgcn_readfirstlane(Rp.lig_ids[li]) : li;
  const bool second = 2 * m + 1 < Rp.kpl;     // the wavefront has two poses
  const int member = 2 * m + (second ? h : 0);
  const bool writer = h == 0 || second;
  const int i = lig * Rp.kpl + member;        // pose index in the caller's layout
  const int abase = __builtin_amdgcn_readfirstlane(P.atom_offset[lig]);
  const int N = __builtin_amdgcn_readfirstlane(P.atom_offset[lig + 1]) - abase;
  const int toff = __builtin_amdgcn_readfirstlane(P.tors_offset[lig]);
  const int K = __builtin_amdgcn_readfirstlane(P.tors_offset[lig + 1]) - toff;
  const size_t cbase = (size_t)Rp.kpl * abase + (size_t)member * N;   // coordinates of the lane's pose
  if (lane < K) {
    tors[lane] = make_int2(P.tors_atoms[2 * (toff + lane)], P.tors_atoms[2 * (toff + lane) + 1]);
    inv_len[lane] = P.inv_len[toff + lane];
  }
  const bool table = axes_fixed_under_torsions(P, abase, toff, K);
  const bool in = la < N;
  PairPose cur, best;
  cur.x[0] = in ? P.x[cbase + la] : 0.f;
  cur.x[1] = in ? P.y[cbase + la] : 0.f;
  cur.x[2] = in ? P.z[cbase + la] : 0.f;
  const uint32_t mk = in ? P.mask[abase + la] : 0u;
  uint32_t mv = mk;   // bonds that rotate the lane's atom (b_k excluded)
  for (int k = 0; k < K; ++k) {
    const int b = __builtin_amdgcn_readfirstlane(P.tors_atoms[2 * (toff + k) + 1]);
    if (la == b) mv &= ~(1u << k);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) cur.piv[d] = P.ref[3 * (size_t)i + d];
  wave_sync();
  best = cur;
  float v = in ? trilinear(G, cur.x[0], cur.x[1], cur.x[2], nullptr) : 0.f;
  float best_s = pair_atom_order_sum(v, N);
  float scale = 1.f;
  float g[6];
  LaneAxis ax{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool fresh = true, pending = false;   // per half, as in refine_kernel
  pair_store_pose(pos_h, cur, mk, N, false);
  wave_sync();
  for (int step = 0; step < Rp.steps; ++step) {
    if (wave_any(fresh)) {
      // both halves take the gradient of their current pose; a half whose pose
      // did not change gets the values it already had
      if (la < K) {
        const int2 t = tors[la];
        const float4 pa = pos_h[t.x], pb = pos_h[t.y];
        const float il = inv_len[la];
        ax = LaneAxis{pa.x, pa.y, pa.z, (pb.x - pa.x) * il, (pb.y - pa.y) * il, (pb.z - pa.z) * il};
      }
      const float sc = pair_move_gradient(G, cur, mk, N, K, tors, pos_h, ax, g, thg_h, tile_h, res_h);
      wave_sync();
      if (pending && sc > best_s) {
        best_s = sc;
        best = cur;
      }
      fresh = pending = false;
    }
    float q[6];
    float dt[3], dw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) { dt[d] = Rp.eta_t * g[d]; dw[d] = Rp.eta_w * g[3 + d]; }
    // clip factors: lane 32 h the translation's, lane 32 h + 1 the rotation's
    float ft, fw;
    {
      const bool rot = la == 1;
      const float a0 = rot ? dw[0] : dt[0], a1 = rot ? dw[1] : dt[1], a2 = rot ? dw[2] : dt[2];
      const float clip = rot ? Rp.clip_w : Rp.clip_t;
      const float nrm = sqrtf(fmaf(a2, a2, fmaf(a1, a1, a0 * a0)));
      const float f = nrm > clip ? clip / nrm : 1.f;
      const float f0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), 0));
      const float f1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), 1));
      const float f32 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), 32));
      const float f33 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f), 33));
      ft = h ? f32 : f0;
      fw = h ? f33 : f1;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      q[d] = (dt[d] * ft) * scale;
      q[3 + d] = (dw[d] * fw) * scale;
    }
    float thk = 0.f;
    if (la < K) {
      float t = Rp.eta_th * thg_h[la];
      t = fminf(fmaxf(t, -Rp.clip_th), Rp.clip_th);
      thk = t * scale;
      th_h[la] = thk;
    }
    PairPose cand = cur;
    const float w2 = fmaf(q[5], q[5], fmaf(q[4], q[4], q[3] * q[3]));
    const bool rot = w2 > 0.f;
    if (table) {
      // lane 32 h + k < K: bond k's matrix of pose h; lane 32 h + K: the rigid rotation's
      float4* mats = reinterpret_cast<float4*>(tile_h);
      float wlen = 0.f, wx = 0.f, wy = 0.f, wz = 0.f;
      if (rot) {
        wlen = sqrtf(w2);
        wx = q[3] / wlen;
        wy = q[4] / wlen;
        wz = q[5] / wlen;
      }
      const bool bond = la < K && thk != 0.f;
      if (bond || (la == K && rot)) {
        const float ang = bond ? thk : wlen;
        const float ux = bond ? ax.ux : wx, uy = bond ? ax.uy : wy, uz = bond ? ax.uz : wz;
        float c, sn, mm[9];
        step_cos_sin(ang, c, sn);
        torsion_matrix(ux, uy, uz, c, sn, mm);
        mats[3 * la] = make_float4(mm[0], mm[1], mm[2], ax.xa);
        mats[3 * la + 1] = make_float4(mm[3], mm[4], mm[5], ax.ya);
        mats[3 * la + 2] = make_float4(mm[6], mm[7], mm[8], ax.za);
      }
      wave_sync();
      for (int k = K - 1; k >= 0; --k) {
        const float ang = th_h[k];
        if (!wave_any(ang != 0.f)) continue;
        if (ang != 0.f && ((mv >> k) & 1u)) {
          const float4 r0 = mats[3 * k], r1 = mats[3 * k + 1], r2 = mats[3 * k + 2];
          const float mm[9] = {r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, r2.x, r2.y, r2.z};
          float y0, y1, y2;
          mat_apply(mm, cand.x[0] - r0.w, cand.x[1] - r1.w, cand.x[2] - r2.w, y0, y1, y2);
          cand.x[0] = r0.w + y0;
          cand.x[1] = r1.w + y1;
          cand.x[2] = r2.w + y2;
        }
      }
      if (rot) {
        const float4 r0 = mats[3 * K], r1 = mats[3 * K + 1], r2 = mats[3 * K + 2];
        const float mm[9] = {r0.x, r0.y, r0.z, r1.x, r1.y, r1.z, r2.x, r2.y, r2.z};
        float y0, y1, y2;
        mat_apply(mm, cand.x[0] - cand.piv[0], cand.x[1] - cand.piv[1], cand.x[2] - cand.piv[2], y0, y1, y2);
        cand.x[0] = cand.piv[0] + y0;
        cand.x[1] = cand.piv[1] + y1;
        cand.x[2] = cand.piv[2] + y2;
      }
    } else {
      // bond axes as they stand when each torsion is applied (reverse order), from
      // the lane's own half
      wave_sync();
      for (int k = K - 1; k >= 0; --k) {
        const float ang = th_h[k];
        if (!wave_any(ang != 0.f)) continue;
        float c, sn;
        step_cos_sin(ang, c, sn);
        const int a = tors[k].x, b = tors[k].y;
        auto pick = [&](float val, int atom) {
          const float v0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(val), atom));
          const float v1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(val), 32 + atom));
          return h ? v1 : v0;
        };
        const float xa = pick(cand.x[0], a), ya = pick(cand.x[1], a), za = pick(cand.x[2], a);
        const float il = inv_len[k];
        const float ux = (pick(cand.x[0], b) - xa) * il, uy = (pick(cand.x[1], b) - ya) * il,
                    uz = (pick(cand.x[2], b) - za) * il;
        float mm[9];
        torsion_matrix(ux, uy, uz, c, sn, mm);
        if (ang != 0.f && ((mv >> k) & 1u)) {
          float y0, y1, y2;
          mat_apply(mm, cand.x[0] - xa, cand.x[1] - ya, cand.x[2] - za, y0, y1, y2);
          cand.x[0] = xa + y0;
          cand.x[1] = ya + y1;
          cand.x[2] = za + y2;
        }
      }
      if (rot) {
        const float wlen = sqrtf(w2);
        float c, sn, mm[9];
        step_cos_sin(wlen, c, sn);
        torsion_matrix(q[3] / wlen, q[4] / wlen, q[5] / wlen, c, sn, mm);
        float y0, y1, y2;
        mat_apply(mm, cand.x[0] - cand.piv[0], cand.x[1] - cand.piv[1], cand.x[2] - cand.piv[2], y0, y1, y2);
        cand.x[0] = cand.piv[0] + y0;
        cand.x[1] = cand.piv[1] + y1;
        cand.x[2] = cand.piv[2] + y2;
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      cand.x[d] = cand.x[d] + q[d];
      cand.piv[d] = cand.piv[d] + q[d];
    }
    wave_sync();
    pair_store_pose(pos_h, cand, mk, N, true);
    wave_sync();
    const bool ok = pair_clash_free(cand, mk, N, tors, pos_h, Rp.clash2);
    wave_sync();
    if (!ok) {
      scale = scale * 0.5f;
      pair_store_pose(pos_h, cur, mk, N, false);   // pos holds the current pose whenever a gradient is due
    } else {
      cur = cand;
      fresh = pending = true;
    }
    wave_sync();
  }
  if (wave_any(pending)) {
    v = in ? trilinear(G, cur.x[0], cur.x[1], cur.x[2], nullptr) : 0.f;
    const float sc = pair_atom_order_sum(v, N);
    if (pending && sc > best_s) {
      best_s = sc;
      best = cur;
    }
  }
  if (writer) {
    if (in) {
      Rp.xo[cbase + la] = best.x[0];
      Rp.yo[cbase + la] = best.x[1];
      Rp.zo[cbase + la] = best.x[2];
    }
    if (la == 0) Rp.score[i] = best_s;
  }
}

// Score of poses moved by given local parameters, and the gradient with respect
// to those parameters: each pose i is moved by q_i = (t, w, theta) (layout of
// lg_score's gradient: 6 i + tors_offset[i]), scored (trilinear, atom order) and
// differentiated.  d/dt and d/dtheta are the force / torque form at the moved
// pose (later moves carry each fragment and its axis rigidly); d/dw is the
// torque about the moved pivot times the transposed left Jacobian of SO(3):
// J^T = I - a [w]x + b [w]x^2, a = (1 - cos|w|)/|w|^2, b = (|w| - sin|w|)/|w|^3.
template <int NSLOT>
__global__ __launch_bounds__(256) void score_moves_kernel(GridDev G, LigDev P, const float* moves, int n,
                                                          float* score, float* grad) {
  extern __shared__ float4 lds[];
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6, lane = lane_id();
  float4* pos = lds + (size_t)wave * (64 * NSLOT + 32 + GRAD_LDS_FLOAT4);
  int2* tors = reinterpret_cast<int2*>(pos + 64 * NSLOT);     // 32 entries
  float* inv_len = reinterpret_cast<float*>(tors + 32);       // 32 entries
  float* th = inv_len + 32;                                   // 32 entries
  float* tile = th + 32;
  float* res = tile + TILE_FLOATS;
  const int i = blockIdx.x * nwaves + wave;
  if (i >= n) return;
  const int abase = __builtin_amdgcn_readfirstlane(P.atom_offset[i]);
  const int N = __builtin_amdgcn_readfirstlane(P.atom_offset[i + 1]) - abase;
  const int toff = __builtin_amdgcn_readfirstlane(P.tors_offset[i]);
  const int K = __builtin_amdgcn_readfirstlane(P.tors_offset[i + 1]) - toff;
  const float* q_i = moves + 6 * (size_t)i + toff;
  if (lane < K) {
    tors[lane] = make_int2(P.tors_atoms[2 * (toff + lane)], P.tors_atoms[2 * (toff + lane) + 1]);
    inv_len[lane] = P.inv_len[toff + lane];
    th[lane] = q_i[6 + lane];
  }
  float q[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) q[d] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(q_i[d])));
  MoveState<NSLOT> p;
  uint32_t mk[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    const bool in = a < N;
    p.x[0][s] = in ? P.x[abase + a] : 0.f;
    p.x[1][s] = in ? P.y[abase + a] : 0.f;
    p.x[2][s] = in ? P.z[abase + a] : 0.f;
    mk[s] = in ? P.mask[abase + a] : 0u;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) p.piv[d] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.ref[3 * i + d])));
  wave_sync();
  apply_move<NSLOT, true>(p, mk, N, K, tors, inv_len, q, th);
  store_pose(pos, p, mk, N);
  float g[6];
  wave_sync();
  const LaneAxis ax = lane_axis(pos, tors, inv_len, K);
  const float sc = move_gradient(G, p, mk, N, K, tors, pos, ax, g, th, tile, res);
  wave_sync();
  if (lane == 0) score[i] = sc;
  if (!grad) return;
  // transposed left Jacobian applied to the torque
  const float w2 = fmaf(q[5], q[5], fmaf(q[4], q[4], q[3] * q[3]));
  float a, b;
  if (w2 < 1e-8f) {
    a = 0.5f - w2 / 24.f;
    b = 1.f / 6.f - w2 / 120.f;
  } else {
    const float w = sqrtf(w2);
    float sn, cs;
    sincosf(w, &sn, &cs);
    a = (1.f - cs) / w2;
    b = (w - sn) / (w2 * w);
  }
  const float tx = g[3], ty = g[4], tz = g[5];
  // [w]x t = w x t ; [w]x^2 t = w x (w x t)
  const float c1x = q[4] * tz - q[5] * ty, c1y = q[5] * tx - q[3] * tz, c1z = q[3] * ty - q[4] * tx;
  const float c2x = q[4] * c1z - q[5] * c1y, c2y = q[5] * c1x - q[3] * c1z, c2z = q[3] * c1y - q[4] * c1x;
  float* out = grad + 6 * (size_t)i + toff;
  if (lane == 0) {
    out[0] = g[0];
    out[1] = g[1];
    out[2] = g[2];
    out[3] = tx - a * c1x + b * c2x;
    out[4] = ty - a * c1y + b * c2y;
    out[5] = tz - a * c1z + b * c2z;
  }
  if (lane < K) out[6 + lane] = th[lane];
}

hipError_t launch_score_moves(int nslot, const GridDev& G, const LigDev& P, const float* moves, int n, float* score,
                              float* grad, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int wpb = 4;
  const dim3 grid((n + wpb - 1) / wpb), block(64 * wpb);
  const size_t lds_bytes = (size_t)wpb * (64 * nslot + 32 + GRAD_LDS_FLOAT4) * sizeof(float4);
  switch (nslot) {
    case 1: hipLaunchKernelGGL(score_moves_kernel<1>, grid, block, lds_bytes, st, G, P, moves, n, score, grad); break;
    case 2: hipLaunchKernelGGL(score_moves_kernel<2>, grid, block, lds_bytes, st, G, P, moves, n, score, grad); break;
    case 3: hipLaunchKernelGGL(score_moves_kernel<3>, grid, block, lds_bytes, st, G, P, moves, n, score, grad); break;
    case 4: hipLaunchKernelGGL(score_moves_kernel<4>, grid, block, lds_bytes, st, G, P, moves, n, score, grad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static size_t refine_lds(int nslot, int wpb) { return (size_t)wpb * refine_wave_float4(nslot) * sizeof(float4); }

// Two poses per wavefront for ligands of at most 32 atoms: n_lig ligands of the
// launch (Rp.lig_ids, or 0..n_lig-1), ceil(kpl / 2) wavefronts each.
hipError_t launch_refine_pair(const GridDev& G, const LigDev& P, const RefineDev& Rp, int n_lig, hipStream_t st) {
  const long long waves = (long long)n_lig * ((Rp.kpl + 1) / 2);
  if (waves == 0) return hipSuccess;
  const int wpb = 4;
  const dim3 grid((unsigned)((waves + wpb - 1) / wpb)), block(64 * wpb);
  const size_t lds_bytes = (size_t)wpb * pair_wave_float4() * sizeof(float4);
  hipLaunchKernelGGL(refine_pair_kernel, grid, block, lds_bytes, st, G, P, Rp, (int)waves);
  return hipGetLastError();
}

hipError_t launch_refine(int nslot, const GridDev& G, const LigDev& P, const RefineDev& Rp, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int wpb = 4;
  const dim3 grid((n + wpb - 1) / wpb), block(64 * wpb);
  switch (nslot) {
    case 1: hipLaunchKernelGGL(refine_kernel<1>, grid, block, refine_lds(1, wpb), st, G, P, Rp, n); break;
    case 2: hipLaunchKernelGGL(refine_kernel<2>, grid, block, refine_lds(2, wpb), st, G, P, Rp, n); break;
    case 3: hipLaunchKernelGGL(refine_kernel<3>, grid, block, refine_lds(3, wpb), st, G, P, Rp, n); break;
    case 4: hipLaunchKernelGGL(refine_kernel<4>, grid, block, refine_lds(4, wpb), st, G, P, Rp, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lg
