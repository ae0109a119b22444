// Pose scoring (nearest / trilinear + force-torque adjoint), pocket padding,
// device-side input preparation (classify / scan / scatter into size buckets)
// and validation kernels.
#include "lg_device.h"

#include <climits>

namespace lg {



// One wavefront per pose: score = sum over atoms in atom order; optional
// gradient with respect to (t, omega, theta) at zero (force / torque form).
__global__ __launch_bounds__(256) void score_kernel(GridDev G, LigDev P, int n, int interp, float* score,
                                                     float* grad) {
  constexpr int NS = 4;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6, lane = lane_id();
  const int i = blockIdx.x * nwaves + wave;
  if (i >= n) return;
  const int abase = __builtin_amdgcn_readfirstlane(P.atom_offset[i]);
  const int N = __builtin_amdgcn_readfirstlane(P.atom_offset[i + 1]) - abase;
  float x[3][NS], g[3][NS], v[NS];
  uint32_t mk[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int a = s * 64 + lane;
    const bool in = a < N;
    x[0][s] = in ? P.x[abase + a] : 0.f;
    x[1][s] = in ? P.y[abase + a] : 0.f;
    x[2][s] = in ? P.z[abase + a] : 0.f;
    mk[s] = in ? P.mask[abase + a] : 0u;
    float gg[3] = {0.f, 0.f, 0.f};
    v[s] = 0.f;
    if (in) v[s] = interp == LG_TRILINEAR ? trilinear(G, x[0][s], x[1][s], x[2][s], gg) : nearest(G, x[0][s], x[1][s], x[2][s]);
    g[0][s] = gg[0]; g[1][s] = gg[1]; g[2][s] = gg[2];
  }
  float total = 0.f;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int cnt = min(64, N - s * 64);
    for (int l = 0; l < cnt; ++l) total = total + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[s]), l));
  }
  if (lane == 0) score[i] = total;
  if (!grad || interp != LG_TRILINEAR) return;
  const int toff = __builtin_amdgcn_readfirstlane(P.tors_offset[i]);
  const int K = __builtin_amdgcn_readfirstlane(P.tors_offset[i + 1]) - toff;
  const float Px = P.ref[3 * i], Py = P.ref[3 * i + 1], Pz = P.ref[3 * i + 2];
  float f[3] = {0.f, 0.f, 0.f}, tq[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    float rx = x[0][s] - Px, ry = x[1][s] - Py, rz = x[2][s] - Pz;
    f[0] += g[0][s]; f[1] += g[1][s]; f[2] += g[2][s];
    tq[0] += ry * g[2][s] - rz * g[1][s];
    tq[1] += rz * g[0][s] - rx * g[2][s];
    tq[2] += rx * g[1][s] - ry * g[0][s];
  }
  float* out = grad + 6 * (size_t)i + toff;
  float red[6];
  for (int c = 0; c < 3; ++c) { red[c] = wave_sum(f[c]); red[3 + c] = wave_sum(tq[c]); }
  if (lane == 0)
    for (int c = 0; c < 6; ++c) out[c] = red[c];
  for (int k = 0; k < K; ++k) {
    const int a = __builtin_amdgcn_readfirstlane(P.tors_atoms[2 * (toff + k)]);
    const int b = __builtin_amdgcn_readfirstlane(P.tors_atoms[2 * (toff + k) + 1]);
    const float xa = atom_value(x[0], a), ya = atom_value(x[1], a), za = atom_value(x[2], a);
    float ux = atom_value(x[0], b) - xa, uy = atom_value(x[1], b) - ya, uz = atom_value(x[2], b) - za;
    const float inv = 1.0f / sqrtf(ux * ux + uy * uy + uz * uz);
    ux *= inv; uy *= inv; uz *= inv;
    float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if ((mk[s] >> k) & 1u) {
        float rx = x[0][s] - xa, ry = x[1][s] - ya, rz = x[2][s] - za;
        t[0] += ry * g[2][s] - rz * g[1][s];
        t[1] += rz * g[0][s] - rx * g[2][s];
        t[2] += rx * g[1][s] - ry * g[0][s];
      }
    }
    const float tk = ux * wave_sum(t[0]) + uy * wave_sum(t[1]) + uz * wave_sum(t[2]);
    if (lane == 0) out[6 + k] = tk;
  }
}

hipError_t launch_score(const GridDev& G, const LigDev& P, int n, int interp, float* score, float* grad,
                        hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int wpb = 4;
  hipLaunchKernelGGL(score_kernel, dim3((n + wpb - 1) / wpb), dim3(64 * wpb), 0, st, G, P, n, interp, score, grad);
  return hipGetLastError();
}

// Copy the grid into the padded layout with an out_value border.
__global__ void pad_kernel(const float* src, int nx, int ny, int nz, float out, float* dst) {
  const long long px = nx + 2, py = ny + 2, pz = nz + 2;
  const long long total = px * py * pz;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long ix = idx % px, iy = (idx / px) % py, iz = idx / (px * py);
    const bool in = ix >= 1 && ix <= nx && iy >= 1 && iy <= ny && iz >= 1 && iz <= nz;
    dst[idx] = in ? src[((iz - 1) * ny + (iy - 1)) * nx + (ix - 1)] : out;
  }
}

// Copy of the padded grid in 4x4x2 bricks (see GridDev); nodes past the padded
// extent (brick round-up) hold out_value and are never addressed.
__global__ void brick_kernel(const float* padded, int px, int py, int pz, int nbx, int nby, int nbz, float out,
                             float* brick) {
  const long long total = (long long)nbx * nby * nbz * 32;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long b = e >> 5;
    const int w = (int)(e & 31);
    const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby), bz = (int)(b / ((long long)nbx * nby));
    const int X = 4 * bx + (w & 3), Y = 4 * by + ((w >> 2) & 3), Z = 2 * bz + (w >> 4);
    brick[e] = (X < px && Y < py && Z < pz) ? padded[((long long)Z * py + Y) * px + X] : out;
  }
}

hipError_t launch_brick(const float* padded, int px, int py, int pz, int nbx, int nby, int nbz, float out,
                        float* brick, hipStream_t st) {
  hipLaunchKernelGGL(brick_kernel, dim3(1024), dim3(256), 0, st, padded, px, py, pz, nbx, nby, nbz, out, brick);
  return hipGetLastError();
}

hipError_t launch_pad(const float* src, int nx, int ny, int nz, float out, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(pad_kernel, dim3(1024), dim3(256), 0, st, src, nx, ny, nz, out, dst);
  return hipGetLastError();
}

// ---------------------------------------------------- input preparation (buckets)
__global__ void zero_kernel(int32_t* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void classify_kernel(const int32_t* atom_offset, const int32_t* tors_offset, int n, ClusterBounds cb,
                                int32_t* cls, int32_t* counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int N = atom_offset[i + 1] - atom_offset[i];
  const int K = tors_offset[i + 1] - tors_offset[i];
  int ca = cb.na - 1, cr = cb.nr - 1;
  for (int c = cb.na - 1; c >= 0; --c)
    if (N <= cb.atom[c]) ca = c;
  for (int c = cb.nr - 1; c >= 0; --c)
    if (K <= cb.rot[c]) cr = c;
  const int b = ca * cb.nr + cr;
  cls[i] = b;
  atomicAdd(&counts[b], 1);
}

__global__ void bucket_scan_kernel(const int32_t* counts, int B, int32_t* start, int32_t* fill) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int s = 0;
    for (int b = 0; b < B; ++b) {
      start[b] = s;
      s += counts[b];
      fill[b] = 0;
    }
    start[B] = s;
  }
}

__global__ void scatter_kernel(const int32_t* cls, int n, const int32_t* start, int32_t* fill, int32_t* perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = cls[i];
  perm[start[b] + atomicAdd(&fill[b], 1)] = i;
}

hipError_t launch_bucketing(const int32_t* atom_offset, const int32_t* tors_offset, int n, const ClusterBounds& cb,
                            int32_t* cls, int32_t* counts, int32_t* start, int32_t* fill, int32_t* perm,
                            int32_t* cursors, hipStream_t st) {
  const int B = cb.na * cb.nr;
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, st, counts, B);
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, st, cursors, B);
  if (n > 0) hipLaunchKernelGGL(classify_kernel, dim3((n + 255) / 256), dim3(256), 0, st, atom_offset, tors_offset, n, cb, cls, counts);
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(64), 0, st, counts, B, start, fill);
  if (n > 0) hipLaunchKernelGGL(scatter_kernel, dim3((n + 255) / 256), dim3(256), 0, st, cls, n, start, fill, perm);
  return hipGetLastError();
}

// ---------------------------------------------------- device validation
// stats: [0] min atoms, [1] max atoms, [2] min bonds, [3] max bonds,
//        [4] count of bad bond ids, [5] count of inconsistent offsets
__global__ void check_kernel(const int32_t* atom_offset, const int32_t* tors_offset, const int32_t* tors_atoms,
                             int n, int total_atoms, int total_tors, int32_t* stats) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a0 = atom_offset[i], a1 = atom_offset[i + 1];
  const int t0 = tors_offset[i], t1 = tors_offset[i + 1];
  const int N = a1 - a0, K = t1 - t0;
  atomicMin(&stats[0], N);
  atomicMax(&stats[1], N);
  atomicMin(&stats[2], K);
  atomicMax(&stats[3], K);
  bool offsets_ok = a0 >= 0 && a1 <= total_atoms && t0 >= 0 && t1 <= total_tors && N >= 0 && K >= 0;
  if (i == 0 && (a0 != 0 || t0 != 0)) offsets_ok = false;
  if (i == n - 1 && (a1 != total_atoms || t1 != total_tors)) offsets_ok = false;
  if (!offsets_ok) {
    atomicAdd(&stats[5], 1);
    return;
  }
  if (tors_atoms)
    for (int k = t0; k < t1; ++k) {
      const int a = tors_atoms[2 * k], b = tors_atoms[2 * k + 1];
      if (a < 0 || a >= N || b < 0 || b >= N || a == b) atomicAdd(&stats[4], 1);
    }
}

__global__ void check_init_kernel(int32_t* stats) {
  if (threadIdx.x == 0) {
    stats[0] = INT_MAX; stats[1] = INT_MIN; stats[2] = INT_MAX; stats[3] = INT_MIN;
    stats[4] = 0; stats[5] = 0;
  }
}

hipError_t launch_check(const int32_t* atom_offset, const int32_t* tors_offset, const int32_t* tors_atoms, int n,
                        int total_atoms, int total_tors, int32_t* stats, hipStream_t st) {
  hipLaunchKernelGGL(check_init_kernel, dim3(1), dim3(64), 0, st, stats);
  if (n > 0)
    hipLaunchKernelGGL(check_kernel, dim3((n + 255) / 256), dim3(256), 0, st, atom_offset, tors_offset, tors_atoms,
                       n, total_atoms, total_tors, stats);
  return hipGetLastError();
}

// ---------------------------------------------------------------- VALU rate probe
// Eight independent chains of non-packed VALU operations per lane, no memory
// traffic but one store per lane: the sustained issue rate of one operation
// (kinds 0-4), of two operations from different chains interleaved (5: v_fma_f32
// and v_add_u32), and of the nearest-node index sequence of a scan sample (6:
// v_add_f32, v_fma_f32, v_med3_f32, v_cvt_flr_i32_f32, v_lshl_add_u32,
// v_add3_u32, v_add_f32; seven VALU operations per step of a chain).
template <int KIND>
__global__ __launch_bounds__(256) void valu_probe_kernel(float* out, int iters, float a, float b) {
  float x[8];
  int y[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    x[i] = threadIdx.x * 0.001f + i;
    y[i] = threadIdx.x + i;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (KIND == 0) x[i] = fmaf(x[i], a, b);                      // v_fma_f32
      if (KIND == 1) x[i] = x[i] + a;                              // v_add_f32
      if (KIND == 2) y[i] = y[i] + it;                             // v_add_u32
      if (KIND == 3) x[i] = __builtin_amdgcn_fmed3f(x[i], a, b);   // v_med3_f32
      if (KIND == 4) y[i] = __mul24(y[i], 3) + it;                 // v_mad_i32_i24
      if (KIND == 5) {
        if (i < 4) x[i] = fmaf(x[i], a, b);
        else y[i] = y[i] + it;
      }
      if (KIND == 6) {
        const float f = __builtin_amdgcn_fmed3f(fmaf(x[i] + a, b, 0.5f), -1.0f, 90.0f);
        int n;
        asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(n) : "v"(f));
        y[i] = (n << 2) + y[i];
        y[i] = y[i] + n + it;
        x[i] = x[i] + (float)(y[i] & 1);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i] + (float)y[i];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_valu_probe(int kind, int blocks, int iters, float* out, hipStream_t st) {
  const dim3 grid(blocks), block(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(valu_probe_kernel<0>, grid, block, 0, st, out, iters, 1.0001f, 0.5f); break;
    case 1: hipLaunchKernelGGL(valu_probe_kernel<1>, grid, block, 0, st, out, iters, 1.0001f, 0.5f); break;
    case 2: hipLaunchKernelGGL(valu_probe_kernel<2>, grid, block, 0, st, out, iters, 1.0001f, 0.5f); break;
    case 3: hipLaunchKernelGGL(valu_probe_kernel<3>, grid, block, 0, st, out, iters, 0.1f, 0.5f); break;
    case 4: hipLaunchKernelGGL(valu_probe_kernel<4>, grid, block, 0, st, out, iters, 0.1f, 0.5f); break;
    case 5: hipLaunchKernelGGL(valu_probe_kernel<5>, grid, block, 0, st, out, iters, 1.0001f, 0.5f); break;
    case 6: hipLaunchKernelGGL(valu_probe_kernel<6>, grid, block, 0, st, out, iters, 1e-7f, 1.0f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lg
