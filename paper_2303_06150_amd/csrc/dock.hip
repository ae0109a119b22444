// Docking kernels for gfx950: restart placement, rigid rotation / translation
// scans, greedy torsion scans with the intramolecular clash check, nearest-voxel
// scan scores, trilinear final score, per-ligand top-k.
//
// Mapping.  One wavefront docks one restart (ligand, r).  A scan's samples are
// spread over the 64 lanes (sample j = lane + 64 q, q < SPL); each lane loops
// over the atoms of the scan, reading per-atom scan data that the wavefront
// staged in LDS (broadcast reads), and accumulates nearest-voxel values
// gathered from the L2-resident grid.  The pose lives in registers, atom
// a = 64 s + lane in slot s < NSLOT.  The best sample comes from a DPP/readlane
// reduction (lowest index among equal scores).  Torsion samples are tested for
// intramolecular clashes in the scoring pass against a pruned list of the
// pairs that can clash at some angle.
//
// Outputs.  Each restart records its final score and the selected sample of
// every scan (a few bytes per scan); the per-ligand top-k then rebuilds the k
// kept poses by replaying their moves with the same apply functions the scans
// use, so the poses are bit-identical to the docked ones without storing every
// restart's coordinates.
//
// Arithmetic contract (matches the CPU oracle bit for bit): FP32, explicit
// fmaf, no contraction; sums of quantised grid values are exact in any order,
// the final trilinear sum runs in atom order.
#include "lg_device.h"

#include <climits>
#include <type_traits>

namespace lg {

template <int NSLOT>
struct PoseReg {
  float x[3][NSLOT];
  float piv[3];
};

template <int SPL>
struct SampleReg {
  float c[SPL], s[SPL], d[SPL];
  uint32_t valid_a, valid_t;   // bit q: sample lane + 64 q exists
  bool half_turn;              // A = 64 SPL and sample j + A/2 is sample j turned by pi:
                               // (cos, sin) of the two are exact negatives
  bool quarter_turn;           // A = 64 SPL and samples j + A/4, j + A/2, j + 3A/4 are j
                               // turned by pi/2, pi, 3pi/2: (-s, c), (-c, -s), (s, -c) exactly
  bool unit;                   // every angle sample has |cos| <= 1 and |sin| <= 1
};





template <int SPL>
__device__ __forceinline__ int wave_argmax(const float (&acc)[SPL], uint32_t alive) {
  const int lane = lane_id();
  int best = INT_MIN, bj = INT_MAX;
#pragma unroll
  for (int q = 0; q < SPL; ++q) {
    int k = orderable(acc[q]);
    if (((alive >> q) & 1u) && k > best) { best = k; bj = lane + 64 * q; }
  }
  int wmax = wave_reduce_i32(best, OpMax());
  return wave_reduce_i32(best == wmax ? bj : INT_MAX, OpMin());
}



// acc[q] += gather(t)[q] over t < n, with the gathers of atom t+1 issued before
// the values of atom t are added (two register buffers, no copies).
template <int Q, int NA, class F>
__device__ __forceinline__ void pipelined_sum(int n, F gather, float (&acc)[NA], int qoff = 0) {
  float v0[Q], v1[Q];
  gather(0, v0);
  int t = 1;
  for (; t + 1 < n; t += 2) {
    gather(t, v1);
    __builtin_amdgcn_sched_barrier(0);   // keep the loads of atom t ahead of the sums of atom t-1
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q + qoff] += v0[q];
    gather(t + 1, v0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q + qoff] += v1[q];
  }
  if (t < n) {
    gather(t, v1);
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q + qoff] += v0[q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q + qoff] += v1[q];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q + qoff] += v0[q];
  }
}

// ---- moves: the selected sample of a scan applied to the pose ----------------
// Rotation by sample j about lab axis E through the pivot.
template <int NSLOT, int E>
__device__ __forceinline__ void apply_rot(const DockDev& D, PoseReg<NSLOT>& p, int j) {
  constexpr int P = (E + 1) % 3, Q = (E + 2) % 3;
  if (j == 0) return;
  const float pP = p.piv[P], pQ = p.piv[Q];
  const float c = D.angles[2 * j], sn = D.angles[2 * j + 1];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    float vp = p.x[P][s] - pP, vq = p.x[Q][s] - pQ;
    float np = fmaf(c, vp, -(sn * vq));
    float nq = fmaf(sn, vp, c * vq);
    p.x[P][s] = pP + np;
    p.x[Q][s] = pQ + nq;
  }
}

// Translation by sample j along lab axis E (the pivot moves along).
template <int NSLOT, int E>
__device__ __forceinline__ void apply_trans(const DockDev& D, PoseReg<NSLOT>& p, int j) {
  if (j == 0) return;
  const int m = j < D.T / 2 ? j : j - D.T;
  const float dd = D.delta * (float)m;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) p.x[E][s] = p.x[E][s] + dd;
  p.piv[E] = p.piv[E] + dd;
  // update the pivot here: left to itself the compiler sinks this add past the
  // torsion scans and keeps dd alive (in scratch) until then
  asm volatile("" : "+v"(p.piv[E]));
}

// Bond k's axis at the current pose: pivot atom a, unit direction u.
struct BondAxis {
  int a, b;
  float xa, ya, za, ux, uy, uz;
};

template <int NSLOT>
__device__ __forceinline__ BondAxis bond_axis(const LigDev& Lg, const PoseReg<NSLOT>& p, int toff, int k) {
  BondAxis A;
  A.a = __builtin_amdgcn_readfirstlane(Lg.tors_atoms[2 * (toff + k)]);
  A.b = __builtin_amdgcn_readfirstlane(Lg.tors_atoms[2 * (toff + k) + 1]);
  const float il = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Lg.inv_len[toff + k])));
  A.xa = atom_value(p.x[0], A.a);
  A.ya = atom_value(p.x[1], A.a);
  A.za = atom_value(p.x[2], A.a);
  const float xb = atom_value(p.x[0], A.b), yb = atom_value(p.x[1], A.b), zb = atom_value(p.x[2], A.b);
  A.ux = (xb - A.xa) * il;
  A.uy = (yb - A.ya) * il;
  A.uz = (zb - A.za) * il;
  return A;
}

// Rotation of the moving fragment of bond k (its atoms other than b) by the
// matrix Mj about the axis through a.
template <int NSLOT>
__device__ __forceinline__ void apply_tors(PoseReg<NSLOT>& p, const BondAxis& A, const float (&Mj)[9],
                                           const bool (&mv)[NSLOT]) {
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    if (mv[s]) {
      float y0, y1, y2;
      mat_apply(Mj, p.x[0][s] - A.xa, p.x[1][s] - A.ya, p.x[2][s] - A.za, y0, y1, y2);
      p.x[0][s] = A.xa + y0;
      p.x[1][s] = A.ya + y1;
      p.x[2][s] = A.za + y2;
    }
  }
}

// Moving atoms of bond k held by this lane: in F_k, not the axis atom b.
template <int NSLOT>
__device__ __forceinline__ void moving_atoms(const uint32_t (&mk)[NSLOT], int N, int k, int b, bool (&mv)[NSLOT]) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int at = s * 64 + lane;
    mv[s] = at < N && ((mk[s] >> k) & 1u) && at != b;
  }
}

// ---- rigid rotation scan about lab axis E through the pivot ------------------
template <int NSLOT, int SPL, int E>
__device__ int rot_scan(const GridDev& G, const DockDev& D, PoseReg<NSLOT>& p, int N, float4* scr,
                        const SampleReg<SPL>& sm, const int* tab) {
  constexpr int P = (E + 1) % 3, Q = (E + 2) % 3;
  const int lane = lane_id();
  const float pP = p.piv[P], pQ = p.piv[Q];
  const float cP = G.c0[P], cQ = G.c0[Q], ih = G.inv_h, fnP = G.fn[P], fnQ = G.fn[Q];
  float s0 = 0.f;
  // With |cos|, |sin| <= 1 a rotated offset is at most |vp| + |vq| per axis
  // (B below covers the rounding of the two products and their sum), and the
  // node map is monotone: when both ends of every atom's range map inside
  // [-1, n], no sample needs the clamp of the node index.
  bool inside = true;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    if (a < N) {
      float vp = p.x[P][s] - pP, vq = p.x[Q][s] - pQ;
      int ie = clamp_node(fmaf(p.x[E][s], G.inv_h, G.c0[E]), G.fn[E]);
      scr[a] = make_float4(vp, vq, __int_as_float(boff(tab + G.tab_base[E] + 1, ie)), 0.f);
      s0 += nearest(G, p.x[0][s], p.x[1][s], p.x[2][s]);
      const float B = (fabsf(vp) + fabsf(vq)) * (1.f + 0x1p-20f);
      inside = inside && fmaf(pP - B, ih, cP) >= -1.f && fmaf(pP + B, ih, cP) <= fnP &&
               fmaf(pQ - B, ih, cQ) >= -1.f && fmaf(pQ + B, ih, cQ) <= fnQ;
    }
  }
  inside = sm.unit && !wave_any(!inside);
  s0 = wave_sum(s0);
  wave_sync();
  float acc[SPL];
#pragma unroll
  for (int q = 0; q < SPL; ++q) acc[q] = 0.f;
  const int* tP = tab + G.tab_base[P] + 1;
  const int* tQ = tab + G.tab_base[Q] + 1;
  const char* gk = G.gk;
  // gathers of atom t+1 are issued before the values of atom t are summed
  auto gather = [&](int t, float (&out)[SPL]) {
    const float4 d = scr[t];
    const int part = __float_as_int(d.z);
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
      float np = fmaf(sm.c[q], d.x, -(sm.s[q] * d.y));
      float nq = fmaf(sm.s[q], d.x, sm.c[q] * d.y);
      float xp = pP + np, xq = pQ + nq;
      int ip = clamp_node(fmaf(xp, ih, cP), fnP);
      int iq = clamp_node(fmaf(xq, ih, cQ), fnQ);
      out[q] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
    }
  };
  // samples j and j + A/2: with (cos, sin) negated the rotated offsets are the
  // exact negatives (fma and products are sign-symmetric), so one 2-D rotation
  // serves both; a zero's sign cannot change the node
  auto gather_half_turn = [&](int t, float (&out)[SPL]) {
    const float4 d = scr[t];
    const int part = __float_as_int(d.z);
#pragma unroll
    for (int q = 0; q < SPL / 2; ++q) {
      float np = fmaf(sm.c[q], d.x, -(sm.s[q] * d.y));
      float nq = fmaf(sm.s[q], d.x, sm.c[q] * d.y);
      int ip = clamp_node(fmaf(pP + np, ih, cP), fnP);
      int iq = clamp_node(fmaf(pQ + nq, ih, cQ), fnQ);
      out[q] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = clamp_node(fmaf(pP - np, ih, cP), fnP);
      iq = clamp_node(fmaf(pQ - nq, ih, cQ), fnQ);
      out[q + SPL / 2] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
    }
  };
  // samples j + A/4 and j + 3A/4 in the same way: with (cos, sin) = (-s, c) the
  // rotated offsets are (-nq, np), with (s, -c) they are (nq, -np), exactly
  auto gather_quarter_turn = [&](int t, float (&out)[SPL]) {
    const float4 d = scr[t];
    const int part = __float_as_int(d.z);
    constexpr int Q4 = SPL / 4;
#pragma unroll
    for (int q = 0; q < Q4; ++q) {
      const float np = fmaf(sm.c[q], d.x, -(sm.s[q] * d.y));
      const float nq = fmaf(sm.s[q], d.x, sm.c[q] * d.y);
      int ip = clamp_node(fmaf(pP + np, ih, cP), fnP);
      int iq = clamp_node(fmaf(pQ + nq, ih, cQ), fnQ);
      out[q] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = clamp_node(fmaf(pP - nq, ih, cP), fnP);
      iq = clamp_node(fmaf(pQ + np, ih, cQ), fnQ);
      out[q + Q4] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = clamp_node(fmaf(pP - np, ih, cP), fnP);
      iq = clamp_node(fmaf(pQ - nq, ih, cQ), fnQ);
      out[q + 2 * Q4] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = clamp_node(fmaf(pP + nq, ih, cP), fnP);
      iq = clamp_node(fmaf(pQ - np, ih, cQ), fnQ);
      out[q + 3 * Q4] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
    }
  };
  // the same, every node index known to lie in range (no clamp)
  auto gather_quarter_turn_inside = [&](int t, float (&out)[SPL]) {
    const float4 d = scr[t];
    const int part = __float_as_int(d.z);
    constexpr int Q4 = SPL / 4;
#pragma unroll
    for (int q = 0; q < Q4; ++q) {
      const float np = fmaf(sm.c[q], d.x, -(sm.s[q] * d.y));
      const float nq = fmaf(sm.s[q], d.x, sm.c[q] * d.y);
      int ip = floor_node(fmaf(pP + np, ih, cP));
      int iq = floor_node(fmaf(pQ + nq, ih, cQ));
      out[q] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = floor_node(fmaf(pP - nq, ih, cP));
      iq = floor_node(fmaf(pQ + np, ih, cQ));
      out[q + Q4] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = floor_node(fmaf(pP - np, ih, cP));
      iq = floor_node(fmaf(pQ - nq, ih, cQ));
      out[q + 2 * Q4] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
      ip = floor_node(fmaf(pP + nq, ih, cP));
      iq = floor_node(fmaf(pQ - np, ih, cQ));
      out[q + 3 * Q4] = grid_at(gk, part + boff(tP, ip) + boff(tQ, iq));
    }
  };
  if (SPL % 4 == 0 && sm.quarter_turn && inside)
    pipelined_sum<SPL>(N, gather_quarter_turn_inside, acc);
  else if (SPL % 4 == 0 && sm.quarter_turn)
    pipelined_sum<SPL>(N, gather_quarter_turn, acc);
  else if (SPL % 2 == 0 && sm.half_turn)
    pipelined_sum<SPL>(N, gather_half_turn, acc);
  else
    pipelined_sum<SPL>(N, gather, acc);
  if (lane == 0) acc[0] = s0;   // sample 0 is the current pose
  const int j = wave_argmax(acc, sm.valid_a);
  apply_rot<NSLOT, E>(D, p, j);
  wave_sync();
  return j;
}

// 32-bit LDS address of a shared-memory pointer, and a float load from one.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p;
}
__device__ __forceinline__ float lds_load(uint32_t addr) {
  return *(const __attribute__((address_space(3))) float*)(uintptr_t)addr;
}

// ---- rigid translation scan along lab axis E ---------------------------------
// A translation moves an atom along E only, so its T samples read nodes of one
// grid line: those between the nodes of the smallest and the largest
// displacement (the node index is monotone in the displacement), span nodes at
// most.  The wavefront reads each atom's run of nodes once -- 64 / span atoms
// per gather instruction, into an LDS stage -- and every sample then takes its
// value from the stage: the same value, node and sum order as a direct gather
// per sample, with a fraction of the gather instructions.  Runs longer than a
// wavefront (very wide translation ranges) fall back to direct gathers, and so
// does STAGE = false (the plain launch, where a lone wavefront per SIMD would
// wait on every group's nodes).
template <int NSLOT, int SPL, int E, bool STAGE>
__device__ int trans_scan(const GridDev& G, const DockDev& D, PoseReg<NSLOT>& p, int N, float4* scr, float* stage,
                          const SampleReg<SPL>& sm, const int* tab) {
  constexpr int P = (E + 1) % 3, Q = (E + 2) % 3;
  const int lane = lane_id();
  const float cE = G.c0[E], ih = G.inv_h, fnE = G.fn[E];
  // displacement delta * m of sample j (m = j, or j - T past T / 2) is monotone in
  // m, so every sample's lies between those of the two extreme m
  const int mlo = D.T >= 2 ? D.T / 2 - D.T : 0, mhi = D.T >= 2 ? D.T / 2 - 1 : 0;
  const float da = D.delta * (float)mlo, db = D.delta * (float)mhi;
  const float dmin = fminf(da, db), dmax = fmaxf(da, db);
  int span = 0;
  bool inside = true;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    if (a < N) {
      int ip = clamp_node(fmaf(p.x[P][s], G.inv_h, G.c0[P]), G.fn[P]);
      int iq = clamp_node(fmaf(p.x[Q][s], G.inv_h, G.c0[Q]), G.fn[Q]);
      const int part = boff(tab + G.tab_base[P] + 1, ip) + boff(tab + G.tab_base[Q] + 1, iq);
      const int lo = clamp_node(fmaf(p.x[E][s] + dmin, ih, cE), fnE);
      const int hi = clamp_node(fmaf(p.x[E][s] + dmax, ih, cE), fnE);
      span = max(span, hi - lo + 1);
      inside = inside && lo >= 0 && hi < G.n[E];   // every sample's f in [0, n): no clamp needed
      scr[a] = make_float4(p.x[E][s], __int_as_float(part), __int_as_float(lo), 0.f);
    }
  }
  span = wave_reduce_i32(span, OpMax());
  inside = !wave_any(!inside);
  wave_sync();
  float acc[SPL];
#pragma unroll
  for (int q = 0; q < SPL; ++q) acc[q] = 0.f;
  const int* tE = tab + G.tab_base[E] + 1;
  const char* gk = G.gk;
  if (!STAGE || span > 64) {
    auto gather = [&](int t, float (&out)[SPL]) {
      const float4 d = scr[t];
      const int part = __float_as_int(d.y);
#pragma unroll
      for (int q = 0; q < SPL; ++q) {
        float xe = d.x + sm.d[q];
        int ie = clamp_node(fmaf(xe, ih, cE), fnE);
        out[q] = grid_at(gk, part + boff(tE, ie));
      }
    };
    pipelined_sum<SPL>(N, gather, acc);
  } else {
    const int per = 64 / span;               // atoms whose runs one gather instruction reads
    const int tt = lane / span, ii = lane - tt * span;
    const int imax = (int)fnE;
    // lane (tt, ii): node lo + ii of atom g * per + tt (clamped into the grid;
    // positions past an atom's own run are never read)
    auto stage_load = [&](int g) {
      const int t = g * per + tt;
      float v = 0.f;
      if (tt < per && t < N) {
        const float4 d = scr[t];
        v = grid_at(gk, __float_as_int(d.y) + boff(tE, min(__float_as_int(d.z) + ii, imax)));
      }
      return v;
    };
    const int groups = (N + per - 1) / per;
    auto staged = [&](auto clamp_tag) {
      constexpr bool CLAMP = decltype(clamp_tag)::value;
      float next = stage_load(0);
      for (int g = 0; g < groups; ++g) {
        float* buf = stage + (g & 1) * 64;    // two buffers: this group's stage is written while
        buf[lane] = next;                     // the previous group's reads are retired
        wave_sync();
        if (g + 1 < groups) next = stage_load(g + 1);
        const int t0 = g * per, t1 = min(N, t0 + per);
        for (int t = t0; t < t1; ++t) {
          const float4 d = scr[t];
          // LDS byte address of the atom's run, shifted so that node ie (in [lo, lo +
          // span)) is at run + 4 ie
          uint32_t run = lds_addr(buf) + 4u * (uint32_t)((t - t0) * span - __float_as_int(d.z));
          asm volatile("" : "+v"(run));   // one base per atom: each sample then adds 4 ie in one shift-add
          int ie[SPL];
          float v[SPL];
#pragma unroll
          for (int q = 0; q < SPL; ++q) {
            const float f = fmaf(d.x + sm.d[q], ih, cE);
            ie[q] = CLAMP ? clamp_node(f, fnE) : floor_node(f);
          }
#pragma unroll
          for (int q = 0; q < SPL; ++q) v[q] = lds_load(run + 4u * (uint32_t)ie[q]);
#pragma unroll
          for (int q = 0; q < SPL; ++q) acc[q] += v[q];
        }
      }
    };
    if (inside)
      staged(std::false_type{});
    else
      staged(std::true_type{});
  }
  const int j = wave_argmax(acc, sm.valid_t);
  apply_trans<NSLOT, E>(D, p, j);
  wave_sync();
  return j;
}

// Square root for the pair prune's radii: the hardware's one-ulp root.  The
// prune only has to keep every pair that can clash, and its 0.05 A margin is
// orders of magnitude above an ulp of a radius (the exact clash test itself
// uses no root).
__device__ __forceinline__ float prune_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Minimum of two floats as one v_min_f32: fminf's quieting of signalling NaNs
// costs two more instructions per call on a loop-carried value.  A NaN operand
// yields the other one, so a NaN distance never counts as a clash, as with the
// comparison d^2 < clash^2.
__device__ __forceinline__ float vmin(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// ---- greedy torsion scan of bond k with the clash check ----------------------
// Admissibility of every sample is decided in the scoring pass.  A moving atom
// sweeps a circle about the bond axis; a (moving, static) pair whose circle never
// comes within clash distance + margin of the static atom cannot clash at any
// angle (the margin is far above the FP32 deviation of the computed rotation from
// the exact circle), so only the remaining "risky" pairs are tested, with the
// oracle's d^2 formula.  The pairs are listed in LDS grouped by moving atom; if
// a scan has more risky pairs than the list holds, the winner is instead tested
// against every pair and dropped while it clashes (same result, slower).
template <int NSLOT, int SPL>
__device__ int tors_scan(const GridDev& G, const LigDev& Lg, const DockDev& D, PoseReg<NSLOT>& p, int N,
                         int toff, int k, const uint32_t* mkl, float4* scr, float4* pairs,
                         const SampleReg<SPL>& sm, const int* tab) {
  constexpr int PAIR_CAP = 128 * NSLOT;
  const int lane = lane_id();
  uint32_t mk[NSLOT];   // fragment masks of this lane's atoms, kept in LDS between scans
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) mk[s] = mkl[s * 64 + lane];
  const BondAxis A = bond_axis(Lg, p, toff, k);
  const int a = A.a, b = A.b;
  const float xa = A.xa, ya = A.ya, za = A.za, ux = A.ux, uy = A.uy, uz = A.uz;

  // moving atoms of F_k other than b, compacted into scr; their current score;
  // axial position h and radius r of every static atom about the bond axis
  bool mv[NSLOT], st[NSLOT];
  float hs[NSLOT], rs[NSLOT];
  int m = 0;
  float s0 = 0.f;
  moving_atoms(mk, N, k, b, mv);
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int at = s * 64 + lane;
    const bool in = at < N;
    const bool inf = in && ((mk[s] >> k) & 1u);
    st[s] = in && !inf && at != a;
    const float vx = p.x[0][s] - xa, vy = p.x[1][s] - ya, vz = p.x[2][s] - za;
    hs[s] = vx * ux + vy * uy + vz * uz;
    rs[s] = prune_sqrt(fmaxf(vx * vx + vy * vy + vz * vz - hs[s] * hs[s], 0.f));
    const uint64_t bal = __ballot(mv[s]);
    const int pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (mv[s]) {
      scr[m + pre] = make_float4(vx, vy, vz, 0.f);
      s0 += nearest(G, p.x[0][s], p.x[1][s], p.x[2][s]);
    }
    m += __popcll(bal);
  }
  s0 = wave_sum(s0);
  wave_sync();

  // risky pairs, grouped by moving atom t; scr[t].w = first pair | count << 16
  int npairs = 0;
  for (int t = 0; t < m; ++t) {
    const float4 v = scr[t];
    const float ht = v.x * ux + v.y * uy + v.z * uz;
    const float rt = prune_sqrt(fmaxf(v.x * v.x + v.y * v.y + v.z * v.z - ht * ht, 0.f));
    const int first = npairs;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const float dh = ht - hs[s], dr = rt - rs[s];
      const bool risky = st[s] && fmaf(dr, dr, dh * dh) < D.clash_r2;
      const uint64_t bal = __ballot(risky);
      const int pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (risky && npairs + pre < PAIR_CAP) pairs[npairs + pre] = make_float4(p.x[0][s], p.x[1][s], p.x[2][s], 0.f);
      npairs += __popcll(bal);
    }
    if (lane == 0) reinterpret_cast<int*>(scr + t)[3] = min(first, PAIR_CAP) | ((npairs - first) << 16);
  }
  const bool overflow = npairs > PAIR_CAP || D.lazy_clash;
  wave_sync();

  float acc[SPL];
#pragma unroll
  for (int q = 0; q < SPL; ++q) acc[q] = 0.f;
  uint32_t clash = 0u;   // bit q: sample lane + 64 q clashes
  constexpr int QG = SPL < 2 ? SPL : 2;   // samples whose matrices are held at once
  const float ih = G.inv_h, clash2 = D.clash2;
  const char* gk = G.gk;
  const int* tX = tab + G.tab_base[0] + 1;
  const int* tY = tab + G.tab_base[1] + 1;
  const int* tZ = tab + G.tab_base[2] + 1;
  if (m > 0) {
#pragma unroll
    for (int g = 0; g < SPL; g += QG) {
      float M[QG][9];
#pragma unroll
      for (int q = 0; q < QG; ++q) torsion_matrix(ux, uy, uz, sm.c[g + q], sm.s[g + q], M[q]);
      auto gather = [&](int t, float (&out)[QG]) {
        const float4 v = scr[t];
        float X[QG], Y[QG], Z[QG];
#pragma unroll
        for (int q = 0; q < QG; ++q) {
          float y0, y1, y2;
          mat_apply(M[q], v.x, v.y, v.z, y0, y1, y2);
          X[q] = xa + y0;
          Y[q] = ya + y1;
          Z[q] = za + y2;
          int ix = clamp_node(fmaf(X[q], ih, G.c0[0]), G.fn[0]);
          int iy = clamp_node(fmaf(Y[q], ih, G.c0[1]), G.fn[1]);
          int iz = clamp_node(fmaf(Z[q], ih, G.c0[2]), G.fn[2]);
          out[q] = grid_at(gk, boff(tX, ix) + boff(tY, iy) + boff(tZ, iz));
        }
        if (!overflow) {
          // the segment is the same on every lane: a scalar loop; the least d^2
          // over the atom's pairs decides its clash bits (min is exact)
          const int seg = __builtin_amdgcn_readfirstlane(__float_as_int(v.w));
          const int p0 = seg & 0xFFFF, p1 = p0 + (seg >> 16);
          if (p1 > p0) {
            float dmin[QG];
#pragma unroll
            for (int q = 0; q < QG; ++q) dmin[q] = __builtin_inff();
            for (int pi = p0; pi < p1; ++pi) {
              const float4 c = pairs[pi];
#pragma unroll
              for (int q = 0; q < QG; ++q) {
                float dx = X[q] - c.x, dy = Y[q] - c.y, dz = Z[q] - c.z;
                dmin[q] = vmin(dmin[q], fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
              }
            }
#pragma unroll
            for (int q = 0; q < QG; ++q)
              if (dmin[q] < clash2) clash |= 1u << (g + q);
          }
        }
      };
      pipelined_sum<QG>(m, gather, acc, g);
    }
  }
  if (lane == 0) {
    acc[0] = s0;        // sample 0 is the current pose,
    clash &= ~1u;       // always admissible
  }

  int j;
  float Mj[9];
  if (!overflow) {
    j = wave_argmax(acc, sm.valid_a & ~clash);
    if (j != 0) torsion_matrix(ux, uy, uz, D.angles[2 * j], D.angles[2 * j + 1], Mj);
  } else {
    // best sample; a winner that clashes is dropped and the next best taken
    float4* cand = pairs;
    uint32_t alive = sm.valid_a;
    for (;;) {
      j = wave_argmax(acc, alive);
      if (j == 0) break;
      torsion_matrix(ux, uy, uz, D.angles[2 * j], D.angles[2 * j + 1], Mj);
      for (int t = lane; t < m; t += 64) {
        const float4 v = scr[t];
        float y0, y1, y2;
        mat_apply(Mj, v.x, v.y, v.z, y0, y1, y2);
        cand[t] = make_float4(xa + y0, ya + y1, za + y2, 0.f);
      }
      wave_sync();
      bool hit = false;
      for (int t = 0; t < m; ++t) {
        const float4 c = cand[t];
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
          float dx = c.x - p.x[0][s], dy = c.y - p.x[1][s], dz = c.z - p.x[2][s];
          float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          hit |= st[s] && d2 < clash2;
        }
      }
      if (!wave_any(hit)) break;
      if (lane == (j & 63)) alive &= ~(1u << (j >> 6));
      wave_sync();
    }
  }
  if (j != 0) apply_tors(p, A, Mj, mv);
  wave_sync();
  return j;
}

template <int SPL>
__device__ void load_samples(const DockDev& D, SampleReg<SPL>& sm) {
  const int lane = lane_id();
  sm.valid_a = 0u;
  sm.valid_t = 0u;
  sm.half_turn = false;
  sm.quarter_turn = false;
#pragma unroll
  for (int q = 0; q < SPL; ++q) {
    const int j = lane + 64 * q;
    if (j < D.A) {
      sm.c[q] = D.angles[2 * j];
      sm.s[q] = D.angles[2 * j + 1];
      sm.valid_a |= 1u << q;
    } else {
      sm.c[q] = 1.f;
      sm.s[q] = 0.f;
    }
    if (j < D.T) {
      const int m = j < D.T / 2 ? j : j - D.T;
      sm.d[q] = D.delta * (float)m;
      sm.valid_t |= 1u << q;
    } else {
      sm.d[q] = 0.f;
    }
  }
  {
    bool u = true;
#pragma unroll
    for (int q = 0; q < SPL; ++q) u = u && fabsf(sm.c[q]) <= 1.f && fabsf(sm.s[q]) <= 1.f;
    sm.unit = !wave_any(!u);
  }
  if (SPL % 2 == 0 && D.A == 64 * SPL) {
    bool pair = true;
#pragma unroll
    for (int q = 0; q < SPL / 2; ++q)
      pair = pair && sm.c[q + SPL / 2] == -sm.c[q] && sm.s[q + SPL / 2] == -sm.s[q];
    sm.half_turn = !wave_any(!pair);
  }
  if (SPL % 4 == 0 && D.A == 64 * SPL) {
    constexpr int Q4 = SPL / 4;
    bool quad = true;
#pragma unroll
    for (int q = 0; q < Q4; ++q)
      quad = quad && sm.c[q + Q4] == -sm.s[q] && sm.s[q + Q4] == sm.c[q] && sm.c[q + 2 * Q4] == -sm.c[q] &&
             sm.s[q + 2 * Q4] == -sm.s[q] && sm.c[q + 3 * Q4] == sm.s[q] && sm.s[q + 3 * Q4] == -sm.c[q];
    sm.quarter_turn = !wave_any(!quad);
  }
}

template <int NSLOT>
struct LigReg {
  int N, K, abase, toff;
  uint32_t mk[NSLOT];
  float P0[3];
};

template <int NSLOT>
__device__ void load_ligand(const LigDev& Lg, int lig, LigReg<NSLOT>& L) {
  const int lane = lane_id();
  L.abase = __builtin_amdgcn_readfirstlane(Lg.atom_offset[lig]);
  L.N = __builtin_amdgcn_readfirstlane(Lg.atom_offset[lig + 1]) - L.abase;
  L.toff = __builtin_amdgcn_readfirstlane(Lg.tors_offset[lig]);
  L.K = __builtin_amdgcn_readfirstlane(Lg.tors_offset[lig + 1]) - L.toff;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int a = s * 64 + lane;
    const bool in = a < L.N;
    L.mk[s] = in ? Lg.mask[L.abase + a] : 0u;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) L.P0[c] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Lg.ref[3 * lig + c])));
}

// The fragment masks of the ligand's atoms into the wavefront's LDS: read by
// every torsion scan, they would otherwise be held in registers through the
// restart loop (and spilled to scratch at the register budget of the persistent
// instances, a store per work item).  Each lane reads back only its own words.
template <int NSLOT>
__device__ __forceinline__ void store_masks(const LigReg<NSLOT>& L, uint32_t* mkl) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) mkl[s * 64 + lane] = L.mk[s];
}

// Restart placement: x = M_r (x0 - P0) + (c + t_r), pivot c + t_r.
template <int NSLOT>
__device__ __forceinline__ void place_pose(const LigDev& Lg, const DockDev& D, const LigReg<NSLOT>& L, int r,
                                           PoseReg<NSLOT>& p) {
  const int lane = lane_id();
  const float* row = D.restarts + 12 * r;
  float m[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) m[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(row[i])));
  float q[3] = {D.c[0] + m[9], D.c[1] + m[10], D.c[2] + m[11]};
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    // the input coordinates are re-read (L2-resident) rather than held in
    // registers, through one 32-bit byte offset on the scalar bases: 64-bit
    // per-lane addresses would be hoisted out of the restart loop and spilled
    const int a = s * 64 + lane;
    const bool in = a < L.N;
    uint32_t off = (uint32_t)(L.abase + a) * 4u;
    asm volatile("" : "+v"(off));   // computed here, per restart
    const float x0 = in ? *reinterpret_cast<const float*>(reinterpret_cast<const char*>(Lg.x) + off) : 0.f;
    const float y0 = in ? *reinterpret_cast<const float*>(reinterpret_cast<const char*>(Lg.y) + off) : 0.f;
    const float z0 = in ? *reinterpret_cast<const float*>(reinterpret_cast<const char*>(Lg.z) + off) : 0.f;
    float vx = x0 - L.P0[0], vy = y0 - L.P0[1], vz = z0 - L.P0[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float y = fmaf(m[3 * c + 2], vz, fmaf(m[3 * c + 1], vy, m[3 * c] * vx));
      p.x[c][s] = y + q[c];
    }
  }
  p.piv[0] = q[0]; p.piv[1] = q[1]; p.piv[2] = q[2];
}

// Selected samples of restart r of a ligand: S rows of 6 + K entries.
__device__ __forceinline__ uint16_t* move_record(const DockDev& D, int lig, int toff, int K, int r) {
  return D.moves + (size_t)D.R * D.S * (6 * (size_t)lig + toff) + (size_t)r * D.S * (6 + K);
}

// One restart: placement, S sweeps, final trilinear score, outputs.
template <int NSLOT, int SPL, bool STAGE = true>
__device__ void dock_restart(const GridDev& G, const LigDev& Lg, const DockDev& D, const SampleReg<SPL>& sm,
                             const LigReg<NSLOT>& L, int lig, int r, float4* scr, float4* cand,
                             const uint32_t* mkl, const int* tab) {
  const int lane = lane_id();
  const int N = L.N;
  PoseReg<NSLOT> p;
  place_pose(Lg, D, L, r, p);

  int16_t* tr = D.trace ? D.trace + ((size_t)lig * D.R + r) * (size_t)D.S * D.trace_w : nullptr;
  uint16_t* mrec = move_record(D, lig, L.toff, L.K, r);
  for (int sw = 0; sw < D.S; ++sw) {
    int jr0 = rot_scan<NSLOT, SPL, 0>(G, D, p, N, scr, sm, tab);
    int jr1 = rot_scan<NSLOT, SPL, 1>(G, D, p, N, scr, sm, tab);
    int jr2 = rot_scan<NSLOT, SPL, 2>(G, D, p, N, scr, sm, tab);
    float* stage = reinterpret_cast<float*>(cand);
    int jt0 = trans_scan<NSLOT, SPL, 0, STAGE>(G, D, p, N, scr, stage, sm, tab);
    int jt1 = trans_scan<NSLOT, SPL, 1, STAGE>(G, D, p, N, scr, stage, sm, tab);
    int jt2 = trans_scan<NSLOT, SPL, 2, STAGE>(G, D, p, N, scr, stage, sm, tab);
    int16_t* trow = tr ? tr + (size_t)sw * D.trace_w : nullptr;
    uint16_t* mrow = mrec + (size_t)sw * (6 + L.K);
    if (lane == 0) {
      mrow[0] = (uint16_t)jr0; mrow[1] = (uint16_t)jr1; mrow[2] = (uint16_t)jr2;
      mrow[3] = (uint16_t)jt0; mrow[4] = (uint16_t)jt1; mrow[5] = (uint16_t)jt2;
    }
    if (trow && lane == 0) {
      trow[0] = (int16_t)jr0; trow[1] = (int16_t)jr1; trow[2] = (int16_t)jr2;
      trow[3] = (int16_t)jt0; trow[4] = (int16_t)jt1; trow[5] = (int16_t)jt2;
    }
    for (int k = 0; k < L.K; ++k) {
      int jk = tors_scan<NSLOT, SPL>(G, Lg, D, p, N, L.toff, k, mkl, scr, cand, sm, tab);
      if (lane == 0) mrow[6 + k] = (uint16_t)jk;
      if (trow && lane == 0) trow[6 + k] = (int16_t)jk;
    }
  }

  // final trilinear score, summed in atom order
  float v[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s)
    v[s] = (s * 64 + lane < N) ? trilinear(G, p.x[0][s], p.x[1][s], p.x[2][s], nullptr) : 0.f;
  float total = 0.f;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int cnt = min(64, N - s * 64);
    for (int l = 0; l < cnt; ++l) total = total + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[s]), l));
  }
  if (lane == 0) D.final_scores[(size_t)lig * D.R + r] = total;
}

// The pose of restart r after its recorded moves: placement, then every
// sweep's rotations, translations and torsions with the selected samples.
template <int NSLOT>
__device__ void replay_restart(const LigDev& Lg, const DockDev& D, const LigReg<NSLOT>& L, int lig, int r,
                               PoseReg<NSLOT>& p) {
  place_pose(Lg, D, L, r, p);
  const uint16_t* mrec = move_record(D, lig, L.toff, L.K, r);
  // recorded indices are below A (rotations, torsions) and T (translations); the
  // clamps only keep table reads in range
  const int amax = D.A - 1, tmax = D.T - 1;
  for (int sw = 0; sw < D.S; ++sw) {
    const uint16_t* mrow = mrec + (size_t)sw * (6 + L.K);
    apply_rot<NSLOT, 0>(D, p, min((int)__builtin_amdgcn_readfirstlane(mrow[0]), amax));
    apply_rot<NSLOT, 1>(D, p, min((int)__builtin_amdgcn_readfirstlane(mrow[1]), amax));
    apply_rot<NSLOT, 2>(D, p, min((int)__builtin_amdgcn_readfirstlane(mrow[2]), amax));
    apply_trans<NSLOT, 0>(D, p, min((int)__builtin_amdgcn_readfirstlane(mrow[3]), tmax));
    apply_trans<NSLOT, 1>(D, p, min((int)__builtin_amdgcn_readfirstlane(mrow[4]), tmax));
    apply_trans<NSLOT, 2>(D, p, min((int)__builtin_amdgcn_readfirstlane(mrow[5]), tmax));
    for (int k = 0; k < L.K; ++k) {
      const int j = min((int)__builtin_amdgcn_readfirstlane(mrow[6 + k]), amax);
      if (j == 0) continue;
      const BondAxis A = bond_axis(Lg, p, L.toff, k);
      float Mj[9];
      torsion_matrix(A.ux, A.uy, A.uz, D.angles[2 * j], D.angles[2 * j + 1], Mj);
      bool mv[NSLOT];
      moving_atoms(L.mk, L.N, k, A.b, mv);
      apply_tors(p, A, Mj, mv);
    }
  }
}

// Plain method: one launch per ligand; wavefront w of the grid docks restart w.
// LDS of a block: the brick offset tables, then per wavefront the scan data of
// 64*NSLOT atoms, a list of 128*NSLOT risky torsion pairs and the fragment masks.
__device__ __forceinline__ int tab_words(const GridDev& G) { return (G.tab_len + 3) & ~3; }

template <int NSLOT, int SPL>
__global__ __launch_bounds__(256) void dock_plain_kernel(GridDev G, LigDev Lg, DockDev D, int lig) {
  extern __shared__ float4 lds[];
  int* tab = reinterpret_cast<int*>(lds);
  fill_brick_tables(G, tab);
  __syncthreads();
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  float4* scr = lds + tab_words(G) / 4 + (size_t)wave * dock_wave_float4(NSLOT);
  float4* cand = scr + 64 * NSLOT;
  uint32_t* mkl = reinterpret_cast<uint32_t*>(scr + 3 * 64 * NSLOT);
  const int r = blockIdx.x * nwaves + wave;
  if (r >= D.R) return;
  SampleReg<SPL> sm;
  load_samples(D, sm);
  LigReg<NSLOT> L;
  load_ligand(Lg, lig, L);
  store_masks(L, mkl);
  // one wavefront per restart: the staged translation scan's read-then-use of
  // each group's nodes would expose their latency, so the gathers stay direct
  dock_restart<NSLOT, SPL, false>(G, Lg, D, sm, L, lig, r, scr, cand, mkl, tab);
}

// Bucketed method: persistent; wavefronts pull (ligand, restart chunk) items of
// one size bucket from an atomic cursor until the bucket is drained.  Occupancy
// target per instance (wavefronts per SIMD), chosen by measurement: the register
// budget it implies makes the compiler spill a few values to scratch, which
// costs less than the latency the extra wavefronts hide.
constexpr int bucket_waves_per_simd(int nslot) { return nslot == 1 ? 6 : nslot == 2 ? 5 : 4; }

template <int NSLOT, int SPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bucket_waves_per_simd(NSLOT))))
void dock_bucket_kernel(GridDev G, LigDev Lg, DockDev D, QueueDev Q) {
  extern __shared__ float4 lds[];
  int* tab = reinterpret_cast<int*>(lds);
  fill_brick_tables(G, tab);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  float4* scr = lds + tab_words(G) / 4 + (size_t)wave * dock_wave_float4(NSLOT);
  float4* cand = scr + 64 * NSLOT;
  uint32_t* mkl = reinterpret_cast<uint32_t*>(scr + 3 * 64 * NSLOT);
  const int lane = lane_id();
  const int b0 = __builtin_amdgcn_readfirstlane(Q.bucket_start[Q.bucket]);
  const int b1 = __builtin_amdgcn_readfirstlane(Q.bucket_start[Q.bucket + 1]);
  const int nch = (D.R + Q.chunk - 1) / Q.chunk;
  const long long n_items = (long long)(b1 - b0) * nch;
  if (n_items == 0) return;
  SampleReg<SPL> sm;
  load_samples(D, sm);
  int cur_lig = -1;
  LigReg<NSLOT> L;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(Q.cursor + Q.bucket, 1);
    item = __builtin_amdgcn_readlane(item, 0);
    if ((long long)item >= n_items) break;
    const int li = item / nch, ch = item - li * nch;
    const int lig = __builtin_amdgcn_readfirstlane(Q.perm[b0 + li]);
    if (lig != cur_lig) {
      load_ligand(Lg, lig, L);
      store_masks(L, mkl);
      cur_lig = lig;
    }
    const int r0 = ch * Q.chunk, r1 = min(D.R, r0 + Q.chunk);
    if (L.N > 64 * NSLOT) {
      // cannot happen with the host's plan (instances sized for the largest
      // ligand); marks the restarts instead of touching memory out of range
      for (int r = r0 + lane; r < r1; r += 64) D.final_scores[(size_t)lig * D.R + r] = __builtin_nanf("");
      continue;
    }
    for (int r = r0; r < r1; ++r) dock_restart(G, Lg, D, sm, L, lig, r, scr, cand, mkl, tab);
  }
}

// Several docking sites: the bucket kernel's loop over items (site, ligand of
// the bucket, restart chunk); each item docks against its site's grid and
// records into the site's scores and moves.  The brick tables depend on the
// grid dimensions only, shared by every site.
template <int NSLOT, int SPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bucket_waves_per_simd(NSLOT))))
void dock_sites_kernel(GridDev G, LigDev Lg, DockDev D, QueueDev Q, SitesDev Sd) {
  extern __shared__ float4 lds[];
  int* tab = reinterpret_cast<int*>(lds);
  fill_brick_tables(G, tab);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  float4* scr = lds + tab_words(G) / 4 + (size_t)wave * dock_wave_float4(NSLOT);
  float4* cand = scr + 64 * NSLOT;
  uint32_t* mkl = reinterpret_cast<uint32_t*>(scr + 3 * 64 * NSLOT);
  const int lane = lane_id();
  const int b0 = __builtin_amdgcn_readfirstlane(Q.bucket_start[Q.bucket]);
  const int b1 = __builtin_amdgcn_readfirstlane(Q.bucket_start[Q.bucket + 1]);
  const int nlig = b1 - b0;
  const int nch = (D.R + Q.chunk - 1) / Q.chunk;
  const long long per_site = (long long)nlig * nch;
  const long long n_items = per_site * Sd.n_sites;
  if (n_items == 0) return;
  SampleReg<SPL> sm;
  load_samples(D, sm);
  int cur_lig = -1;
  LigReg<NSLOT> L;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(Q.cursor + Q.bucket, 1);
    item = __builtin_amdgcn_readlane(item, 0);
    if ((long long)item >= n_items) break;
    int site, li, ch;
    if (Sd.site_major) {
      site = (int)(item / per_site);
      const int rem = (int)(item - site * per_site);
      li = rem / nch;
      ch = rem - li * nch;
    } else {
      li = item / (nch * Sd.n_sites);
      const int rem = item - li * nch * Sd.n_sites;
      site = rem / nch;
      ch = rem - site * nch;
    }
    const int lig = __builtin_amdgcn_readfirstlane(Q.perm[b0 + li]);
    if (lig != cur_lig) {
      load_ligand(Lg, lig, L);
      store_masks(L, mkl);
      cur_lig = lig;
    }
    // the site's fields as uniform words: a plain load of Sd.grids would be
    // held in vector registers for the whole item
    GridDev Gs = G;
    DockDev Ds = D;
    {
      const int* w = reinterpret_cast<const int*>(Sd.grids + site);
      int v[sizeof(SiteGrid) / 4];
#pragma unroll
      for (int k = 0; k < (int)(sizeof(SiteGrid) / 4); ++k) v[k] = __builtin_amdgcn_readfirstlane(w[k]);
      SiteGrid sg;
      __builtin_memcpy(&sg, v, sizeof sg);
      Gs.g0 = sg.g0;
      Gs.gb = sg.gb;
      Gs.gk = sg.gk;
      for (int a = 0; a < 3; ++a) {
        Gs.c0[a] = sg.c0[a];
        Gs.o[a] = sg.o[a];
      }
      Gs.out = sg.out;
      for (int a = 0; a < 3; ++a) Ds.c[a] = sg.c[a];
    }
    Ds.final_scores = D.final_scores + (size_t)site * Sd.scores_stride;
    Ds.moves = D.moves + (size_t)site * Sd.moves_stride;
    const int r0 = ch * Q.chunk, r1 = min(D.R, r0 + Q.chunk);
    if (L.N > 64 * NSLOT) {
      for (int r = r0 + lane; r < r1; r += 64) Ds.final_scores[(size_t)lig * D.R + r] = __builtin_nanf("");
      continue;
    }
    for (int r = r0; r < r1; ++r) dock_restart(Gs, Lg, Ds, sm, L, lig, r, scr, cand, mkl, tab);
  }
}

// Per-ligand top-k over restarts (score descending, equal scores: lower r);
// the kept poses and pivots rebuilt from their recorded moves.  One wavefront
// per ligand.
template <int NSLOT>
__global__ __launch_bounds__(256) void topk_kernel(LigDev Lg, DockDev D, int n, int k, float* score,
                                                    int32_t* rid, float* ox, float* oy, float* oz,
                                                    float* all_scores, float* opiv) {
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6, lane = lane_id();
  const int lig = blockIdx.x * nwaves + wave;
  if (lig >= n) return;
  const float* fs = D.final_scores + (size_t)lig * D.R;
  if (all_scores)
    for (int r = lane; r < D.R; r += 64) all_scores[(size_t)lig * D.R + r] = fs[r];
  LigReg<NSLOT> L;
  load_ligand(Lg, lig, L);
  if (L.N > 64 * NSLOT) return;   // cannot happen: the instance is sized for the largest ligand
  int pk = INT_MAX, pr = -1;   // previous selection (key, r)
  for (int qi = 0; qi < k; ++qi) {
    int best = INT_MIN, br = INT_MAX;
    for (int r = lane; r < D.R; r += 64) {
      const int key = orderable(fs[r] + 0.0f);
      const bool after = key < pk || (key == pk && r > pr);
      if (after && (key > best || (key == best && r < br))) { best = key; br = r; }
    }
    const int wmax = wave_reduce_i32(best, OpMax());
    const int rs = wave_reduce_i32(best == wmax ? br : INT_MAX, OpMin());
    pk = wmax;
    pr = rs;
    if (lane == 0) {
      score[(size_t)lig * k + qi] = fs[rs];
      rid[(size_t)lig * k + qi] = rs;
    }
    PoseReg<NSLOT> p;
    replay_restart(Lg, D, L, lig, rs, p);
    const size_t dst = (size_t)k * L.abase + (size_t)qi * L.N;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int a = s * 64 + lane;
      if (a < L.N) {
        ox[dst + a] = p.x[0][s];
        oy[dst + a] = p.x[1][s];
        oz[dst + a] = p.x[2][s];
      }
    }
    const float pv = lane == 0 ? p.piv[0] : lane == 1 ? p.piv[1] : p.piv[2];
    if (opiv && lane < 3) opiv[((size_t)lig * k + qi) * 3 + lane] = pv;
  }
}

// ---------------------------------------------------------------- dispatch
// LDS per block: the brick offset tables, then per wavefront the scan data,
// torsion candidates and fragment masks of 64*NSLOT atoms.
static size_t lds_bytes(int nslot, int wpb, int tab_len) {
  return (size_t)((tab_len + 3) & ~3) * sizeof(int) + (size_t)wpb * dock_wave_float4(nslot) * sizeof(float4);
}

#define LG_DISPATCH(nslot, spl, CALL)                                          \
  switch (nslot * 100 + spl) {                                                 \
    case 101: CALL(1, 1); case 102: CALL(1, 2); case 104: CALL(1, 4);          \
    case 108: CALL(1, 8); case 116: CALL(1, 16);                               \
    case 201: CALL(2, 1); case 202: CALL(2, 2); case 204: CALL(2, 4);          \
    case 208: CALL(2, 8); case 216: CALL(2, 16);                               \
    case 301: CALL(3, 1); case 302: CALL(3, 2); case 304: CALL(3, 4);          \
    case 308: CALL(3, 8); case 316: CALL(3, 16);                               \
    case 401: CALL(4, 1); case 402: CALL(4, 2); case 404: CALL(4, 4);          \
    case 408: CALL(4, 8); case 416: CALL(4, 16);                               \
    default: return hipErrorInvalidValue;                                      \
  }

hipError_t launch_dock_plain(int nslot, int spl, int wpb, const GridDev& G, const LigDev& Lg, const DockDev& D,
                             int lig, hipStream_t st) {
  const int blocks = (D.R + wpb - 1) / wpb;
#define CALL(NS, SP)                                                                            \
  {                                                                                             \
    hipLaunchKernelGGL((dock_plain_kernel<NS, SP>), dim3(blocks), dim3(64 * wpb),               \
                       lds_bytes(NS, wpb, G.tab_len), st, G, Lg, D, lig);                              \
    return hipGetLastError();                                                                   \
  }
  LG_DISPATCH(nslot, spl, CALL)
#undef CALL
}

hipError_t launch_dock_bucket(int nslot, int spl, int wpb, int blocks, const GridDev& G, const LigDev& Lg,
                              const DockDev& D, const QueueDev& Q, hipStream_t st) {
#define CALL(NS, SP)                                                                            \
  {                                                                                             \
    hipLaunchKernelGGL((dock_bucket_kernel<NS, SP>), dim3(blocks), dim3(64 * wpb),              \
                       lds_bytes(NS, wpb, G.tab_len), st, G, Lg, D, Q);                                \
    return hipGetLastError();                                                                   \
  }
  LG_DISPATCH(nslot, spl, CALL)
#undef CALL
}

hipError_t launch_dock_sites(int nslot, int spl, int wpb, int blocks, const GridDev& G, const LigDev& Lg,
                             const DockDev& D, const QueueDev& Q, const SitesDev& Sd, hipStream_t st) {
#define CALL(NS, SP)                                                                            \
  {                                                                                             \
    hipLaunchKernelGGL((dock_sites_kernel<NS, SP>), dim3(blocks), dim3(64 * wpb),               \
                       lds_bytes(NS, wpb, G.tab_len), st, G, Lg, D, Q, Sd);                     \
    return hipGetLastError();                                                                   \
  }
  LG_DISPATCH(nslot, spl, CALL)
#undef CALL
}

// Resident blocks per compute unit of a bucket kernel instance (the b of Eq. 1).
hipError_t occupancy_dock_bucket(int nslot, int spl, int wpb, int tab_len, int* blocks_per_cu) {
#define CALL(NS, SP)                                                                                  \
  {                                                                                                   \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, dock_bucket_kernel<NS, SP>,    \
                                                        64 * wpb, lds_bytes(NS, wpb, tab_len));            \
  }
  LG_DISPATCH(nslot, spl, CALL)
#undef CALL
}

hipError_t attributes_dock_bucket(int nslot, int spl, hipFuncAttributes* attr) {
#define CALL(NS, SP) \
  { return hipFuncGetAttributes(attr, reinterpret_cast<const void*>(dock_bucket_kernel<NS, SP>)); }
  LG_DISPATCH(nslot, spl, CALL)
#undef CALL
}

hipError_t launch_topk(int nslot, const LigDev& Lg, const DockDev& D, int n, int k, float* score, int32_t* rid,
                       float* ox, float* oy, float* oz, float* all_scores, float* pivot, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int wpb = 4;
  const dim3 grid((n + wpb - 1) / wpb), block(64 * wpb);
  switch (nslot) {
    case 1: hipLaunchKernelGGL(topk_kernel<1>, grid, block, 0, st, Lg, D, n, k, score, rid, ox, oy, oz, all_scores, pivot); break;
    case 2: hipLaunchKernelGGL(topk_kernel<2>, grid, block, 0, st, Lg, D, n, k, score, rid, ox, oy, oz, all_scores, pivot); break;
    case 3: hipLaunchKernelGGL(topk_kernel<3>, grid, block, 0, st, Lg, D, n, k, score, rid, ox, oy, oz, all_scores, pivot); break;
    case 4: hipLaunchKernelGGL(topk_kernel<4>, grid, block, 0, st, Lg, D, n, k, score, rid, ox, oy, oz, all_scores, pivot); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lg
