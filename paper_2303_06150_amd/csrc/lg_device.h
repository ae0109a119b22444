// Device helpers shared by the docking, scoring and refinement kernels: grid
// lookups (nearest node on the padded grid, trilinear with gradient), values of
// register-resident atoms, the rotation-matrix script of the scans, and the
// (cos, sin) polynomial of refinement steps.
#pragma once
#include "lg_internal.h"

namespace lg {

__device__ __forceinline__ int node_off(const GridDev& G, float x, float y, float z) {
  int ix = clamp_node(fmaf(x, G.inv_h, G.c0[0]), G.fn[0]);
  int iy = clamp_node(fmaf(y, G.inv_h, G.c0[1]), G.fn[1]);
  int iz = clamp_node(fmaf(z, G.inv_h, G.c0[2]), G.fn[2]);
  return mad24(ix, G.bs[0], mad24(iy, G.bs[1], mad24(iz, G.bs[2], G.b0)));
}

// Brick byte offset of node index i in [-1, n] from an axis table (t = tab + base + 1).
__device__ __forceinline__ int boff(const int* t, int i) { return t[i]; }

__device__ __forceinline__ float nearest(const GridDev& G, float x, float y, float z) {
  return grid_at(G.gb, node_off(G, x, y, z));
}

// Trilinear value (and gradient if g != nullptr); same op order as the oracle.
__device__ __forceinline__ float trilinear(const GridDev& G, float x, float y, float z, float* g) {
  float f0 = (x - G.o[0]) * G.inv_h, f1 = (y - G.o[1]) * G.inv_h, f2 = (z - G.o[2]) * G.inv_h;
  bool in = f0 >= 0.f && f0 < G.fn1[0] && f1 >= 0.f && f1 < G.fn1[1] && f2 >= 0.f && f2 < G.fn1[2];
  if (!in) {
    if (g) g[0] = g[1] = g[2] = 0.f;
    return G.out;
  }
  int i0 = (int)f0, i1 = (int)f1, i2 = (int)f2;
  float w0 = f0 - (float)i0, w1 = f1 - (float)i1, w2 = f2 - (float)i2;
  const int s1 = G.stride[1], s2 = G.stride[2];
  const float* p = G.g0 + i0 + i1 * s1 + i2 * s2;
  float c000 = p[0], c100 = p[1], c010 = p[s1], c110 = p[s1 + 1];
  float c001 = p[s2], c101 = p[s2 + 1], c011 = p[s2 + s1], c111 = p[s2 + s1 + 1];
  float c00 = fmaf(w0, c100 - c000, c000), c10 = fmaf(w0, c110 - c010, c010);
  float c01 = fmaf(w0, c101 - c001, c001), c11 = fmaf(w0, c111 - c011, c011);
  float c0 = fmaf(w1, c10 - c00, c00), c1 = fmaf(w1, c11 - c01, c01);
  float v = fmaf(w2, c1 - c0, c0);
  if (g) {
    float e00 = c100 - c000, e10 = c110 - c010, e01 = c101 - c001, e11 = c111 - c011;
    float e0 = fmaf(w1, e10 - e00, e00), e1 = fmaf(w1, e11 - e01, e01);
    g[0] = fmaf(w2, e1 - e0, e0) * G.inv_h;
    float d0 = c10 - c00, d1 = c11 - c01;
    g[1] = fmaf(w2, d1 - d0, d0) * G.inv_h;
    g[2] = (c1 - c0) * G.inv_h;
  }
  return v;
}

// Value of register array v for atom a, taken from the lane that holds it.
template <int NSLOT>
__device__ __forceinline__ float atom_value(const float (&v)[NSLOT], int a) {
  // one readlane per slot, selected on the scalar side (no dynamic register index)
  const int slot = a >> 6, l = a & 63;
  int r = __builtin_amdgcn_readlane(__float_as_int(v[0]), l);
#pragma unroll
  for (int s = 1; s < NSLOT; ++s) {
    const int rs = __builtin_amdgcn_readlane(__float_as_int(v[s]), l);
    r = slot == s ? rs : r;
  }
  return __int_as_float(r);
}

__device__ __forceinline__ void torsion_matrix(float ux, float uy, float uz, float c, float s, float m[9]) {
  float t = 1.0f - c;
  float tx = t * ux, ty = t * uy, tz = t * uz;
  m[0] = fmaf(tx, ux, c);
  m[4] = fmaf(ty, uy, c);
  m[8] = fmaf(tz, uz, c);
  m[1] = fmaf(tx, uy, -(s * uz));
  m[3] = fmaf(tx, uy, s * uz);
  m[2] = fmaf(tx, uz, s * uy);
  m[6] = fmaf(tx, uz, -(s * uy));
  m[5] = fmaf(ty, uz, -(s * ux));
  m[7] = fmaf(ty, uz, s * ux);
}

__device__ __forceinline__ void mat_apply(const float m[9], float vx, float vy, float vz, float& y0, float& y1,
                                          float& y2) {
  y0 = fmaf(m[2], vz, fmaf(m[1], vy, m[0] * vx));
  y1 = fmaf(m[5], vz, fmaf(m[4], vy, m[3] * vx));
  y2 = fmaf(m[8], vz, fmaf(m[7], vy, m[6] * vx));
}

// (cos x, sin x) for |x| <= pi/4 (refinement steps are clipped to that range):
// Taylor series to x^13 / x^12, Horner in x^2 with fmaf -- the same polynomial the
// CPU reference evaluates.
__device__ __forceinline__ void step_cos_sin(float x, float& c, float& s) {
  const float x2 = x * x;
  float ps = (float)(1.0 / 6227020800.0);
  ps = fmaf(ps, x2, (float)(-1.0 / 39916800.0));
  ps = fmaf(ps, x2, (float)(1.0 / 362880.0));
  ps = fmaf(ps, x2, (float)(-1.0 / 5040.0));
  ps = fmaf(ps, x2, (float)(1.0 / 120.0));
  ps = fmaf(ps, x2, (float)(-1.0 / 6.0));
  s = fmaf(x * x2, ps, x);
  float pc = (float)(1.0 / 479001600.0);
  pc = fmaf(pc, x2, (float)(-1.0 / 3628800.0));
  pc = fmaf(pc, x2, (float)(1.0 / 40320.0));
  pc = fmaf(pc, x2, (float)(-1.0 / 720.0));
  pc = fmaf(pc, x2, (float)(1.0 / 24.0));
  pc = fmaf(pc, x2, -0.5f);
  c = fmaf(x2, pc, 1.0f);
}

// Sum of v over atoms 0..N-1 in atom order (atom 64 s + lane in slot s); the
// result is uniform.
template <int NSLOT>
__device__ __forceinline__ float atom_order_sum(const float (&v)[NSLOT], int N) {
  float total = 0.f;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int cnt = min(64, N - s * 64);
    for (int l = 0; l < cnt; ++l) total = total + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[s]), l));
  }
  return total;
}

}  // namespace lg
