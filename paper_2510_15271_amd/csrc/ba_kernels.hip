// gfx950 kernels of the Levenberg-Marquardt bundle-adjustment iteration.
//
// Math (paper Sec. 4.3): residual r = pi(K (R X + t)) - z of one observation,
// cost 1/2 sum rho(||r||^2) with Huber rho on the squared norm, left SE(3)
// increments.  Per LM iteration, for every problem of a batch:
//
//   linearize    obs-parallel, point tiles: r, Huber weight, sqrt(w)-scaled
//                J_c (2x6) and J_p (2x3) stored per observation; V_j, g_p,j
//                and the cost reduced per point / per tile without atomics.
//   point_prep   V*_j = V_j + lambda D_j inverted (FP64), Y_k = W_k V*_j^-1.
//   schur_diag   one workgroup per free camera a: U_a, g_c,a, the diagonal
//                block S_aa = U*_a - sum Y W^T, b_a = -g_c,a + sum Y g_p, the
//                FP64 6x6 inverse of S_aa (block-Jacobi) and the PCG start.
//   schur_off    one wavefront per upper block S_ab: sum over the points seen
//                by a and b of -Y_aj W_bj^T from precomputed pair lists, one
//                wave reduction, written to S_ab and its transpose.
//   cg_start /   block-Jacobi PCG in its one-reduction form, one launch per
//   cg_step      iteration: block-sparse S u over the columns a tile reads,
//                FP64 dot products from per-tile partials reduced in a fixed
//                order by every consumer -- no grid barrier, no float atomics.
//                (pcg_spmv / pcg_update: the textbook form, two launches per
//                iteration, for systems whose tile columns exceed LDS.)
//   cam_update   T <- Exp(dc) T, camera part of the predicted decrease.
//   point_trial  dp_j = V*_j^-1 (-g_p,j - sum W^T dc), X <- X + dp, trial cost.
//   lm_control   gain ratio, accept/reject, Nielsen damping update.
//
// Every reduction is deterministic: a fixed assignment of work to lanes and a
// fixed summation order, so a problem's result is the same whichever other
// problems share its launches.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cstdint>

#include "ba_internal.h"

namespace bax {

const char *const kKernelNames[K_NUM_KERNELS] = {
    "linearize", "point_prep", "schur_diag", "schur_off", "pcg_spmv", "pcg_update",
    "cam_update", "point_trial", "lm_control", "eval", "pose_gn", "pcg_cg", "schur_chunk",
    "schur_reduce", "schur_rows", "schur_finish", "prior_lin", "prior_apply", "cull", "rig_blocks",
    "rig_rows", "rig_update", "prior_cost", "dense_prep", "dense_cams", "dense_schur", "dense_reduce"};

// A pointer read from a problem's device view is generic to the compiler, which then
// issues flat memory instructions; a flat access also counts against the LDS wait
// counter, so an LDS read waits for every such access still in flight.  Accesses made
// through as_global(p) are global ones.
template <class T>
using global_t = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ global_t<T> *as_global(T *p) {
  return (global_t<T> *)p;
}

// ------------------------------------------------------------------ storage codecs
// Jacobians are stored scaled by sqrt(w).  FP16 storage keeps them times 2^-4 so
// that entries up to 1e6 stay finite; BF16 has the FP32 exponent range.
struct bf16s {
  uint16_t b;
};

template <class S>
struct Codec;
template <>
struct Codec<double> {
  __device__ static double enc(double v) { return v; }
  __device__ static double dec(double v) { return v; }
};
template <>
struct Codec<float> {
  __device__ static float enc(float v) { return v; }
  __device__ static float dec(float v) { return v; }
};
template <>
struct Codec<_Float16> {
  __device__ static _Float16 enc(float v) { return (_Float16)(v * 0.0625f); }
  __device__ static float dec(_Float16 h) { return (float)h * 16.0f; }
};
template <>
struct Codec<bf16s> {
  __device__ static bf16s enc(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16s{(uint16_t)(u >> 16)};  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return bf16s{(uint16_t)(u >> 16)};
  }
  __device__ static float dec(bf16s h) { return __uint_as_float((uint32_t)h.b << 16); }
};

// Linearisation record of one observation, kept compact: the four non-zero
// entries of sqrt(w) J_pi (fx/z, -fx x/z^2, fy/z, -fy y/z^2, each times sqrt(w))
// and the camera-frame point P_c = (x, y, z).  J_c = J_pi [I | -[P]x] and
// J_p = J_pi R are rebuilt from them, R being the camera's rotation.
template <class T, class S>
struct LinRec {
  S f[7];
  T e[2];  // sqrt(w) r
};

// A record between registers and global memory, as 32-bit words.
template <class R>
__device__ __forceinline__ R load_rec(const global_t<const R> *p) {
  static_assert(sizeof(R) % 4 == 0, "records are whole words");
  R r;
  const auto w = (const global_t<const uint32_t> *)p;
  uint32_t *d = reinterpret_cast<uint32_t *>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(R) / 4); ++i) d[i] = w[i];
  return r;
}
template <class R>
__device__ __forceinline__ void store_rec(global_t<R> *p, const R &r) {
  const auto w = (global_t<uint32_t> *)p;
  const uint32_t *d = reinterpret_cast<const uint32_t *>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(R) / 4); ++i) w[i] = d[i];
}

template <class T, class S>
__device__ inline void decode(const LinRec<T, S> &rec, T f[7]) {
#pragma unroll
  for (int i = 0; i < 7; ++i) f[i] = Codec<S>::dec(rec.f[i]);
}

// J_c (2x6, row-major) from the compact record.
template <class T>
__device__ inline void jc_from(const T f[7], T Jc[12]) {
  const T a = f[0], b = f[1], c = f[2], d = f[3], x = f[4], y = f[5], z = f[6];
  Jc[0] = a;     Jc[1] = T(0);  Jc[2] = b;
  Jc[3] = b * y; Jc[4] = a * z - b * x; Jc[5] = -a * y;
  Jc[6] = T(0);  Jc[7] = c;     Jc[8] = d;
  Jc[9] = -c * z + d * y; Jc[10] = -d * x; Jc[11] = c * x;
}

// J_p (2x3, row-major) = J_pi R.
template <class T>
__device__ inline void jp_from(const T f[4], const T R[9], T Jp[6]) {
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Jp[m] = f[0] * R[m] + f[1] * R[6 + m];
    Jp[3 + m] = f[2] * R[3 + m] + f[3] * R[6 + m];
  }
}

// Products with the camera Jacobian.  Each of its two rows holds a structural zero
// (row 0 at column 1, row 1 at column 0, see jc_from); the products below skip those
// terms and accumulate through chains of fused multiply-adds, acc = fma(x, y, acc),
// instead of forming each two-term sum first and adding it.
template <class T>
__device__ inline T fmac(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}

// z = J_c^T m for the 2x2 m = [m00 m01; m10 m11]: z0 its first column, z1 its second.
template <class T>
__device__ inline void jct_m(const T Jc[12], T m00, T m01, T m10, T m11, T z0[6], T z1[6]) {
  z0[0] = Jc[0] * m00;
  z1[0] = Jc[0] * m01;
  z0[1] = Jc[7] * m10;
  z1[1] = Jc[7] * m11;
#pragma unroll
  for (int r = 2; r < 6; ++r) {
    z0[r] = fmac(Jc[6 + r], m10, Jc[r] * m00);
    z1[r] = fmac(Jc[6 + r], m11, Jc[r] * m01);
  }
}

// acc (6x6, row-major) += [z0 z1] J_b for a 6x2 left factor.
template <class T>
__device__ inline void acc_zj(T acc[36], const T z0[6], const T z1[6], const T Jb[12]) {
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      T v = acc[6 * r + c];
      if (c != 1) v = fmac(z0[r], Jb[c], v);
      if (c != 0) v = fmac(z1[r], Jb[6 + c], v);
      acc[6 * r + c] = v;
    }
}

// acc (upper triangle of a 6x6, rows in order, 21 values) += [z0 z1] J_b.
template <class T>
__device__ inline void acc_zj_upper(T acc[21], const T z0[6], const T z1[6], const T Jb[12]) {
  int u = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c, ++u) {
      T v = acc[u];
      if (c != 1) v = fmac(z0[r], Jb[c], v);
      if (c != 0) v = fmac(z1[r], Jb[6 + c], v);
      acc[u] = v;
    }
}

// acc (upper triangle, 21 values) += J_c^T J_c; the (0, 1) element is zero for
// every observation and is left as it is.
template <class T>
__device__ inline void acc_jtj_upper(T acc[21], const T Jc[12]) {
  int u = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c, ++u) {
      T v = acc[u];
      if (r != 1 && c != 1) v = fmac(Jc[r], Jc[c], v);
      if (r != 0 && c != 0) v = fmac(Jc[6 + r], Jc[6 + c], v);
      acc[u] = v;
    }
}

template <class T>
__device__ inline void load_rot(const global_t<const double> *pose, T R[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = T(pose[i]);
}
template <class T>
__device__ inline void load_rot(const double *pose, T R[9]) {  // pose: a pose buffer in global memory
  load_rot(as_global(pose), R);
}

size_t lin_record_bytes(int precision) {
  switch (precision) {
    case 0: return sizeof(LinRec<double, double>);
    case 1: return sizeof(LinRec<float, float>);
    case 2: return sizeof(LinRec<float, _Float16>);
    default: return sizeof(LinRec<float, bf16s>);
  }
}
size_t compute_bytes(int precision) { return precision == 0 ? 8 : 4; }

// ------------------------------------------------------------------ small helpers
template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds one pass of kObsChunk observations' NV values (c; jl = their point in the
// tile, -1 for none) into the points' accumulators s_acc.  The observations of one
// point are consecutive, so an inclusive
// segmented scan across each wave (six shuffle steps) leaves every wave's part of a
// point at its last lane; the chunk's last lane of the point then adds the point's
// wave parts in wave order.  s_c and s_loc are scratch of kObsChunk rows.
template <class T, int NV>
__device__ inline void seg_add_scan(T c[NV], int jl, T (*s_acc)[NV], T (*s_c)[NV], int *s_loc) {
  const int t = threadIdx.x, lane = t & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int oj = __shfl_up(jl, d, 64);
    T o[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) o[i] = __shfl_up(c[i], d, 64);
    if (lane >= d && oj == jl)
#pragma unroll
      for (int i = 0; i < NV; ++i) c[i] += o[i];
  }
  s_loc[t] = jl;
#pragma unroll
  for (int i = 0; i < NV; ++i) s_c[t][i] = c[i];
  __syncthreads();
  if (jl >= 0 && (t == kObsChunk - 1 || s_loc[t + 1] != jl)) {
    const int w = t >> 6;
    int w0 = w;
    while (w0 > 0 && s_loc[(w0 << 6) - 1] == jl) --w0;
    T tot[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) tot[i] = w0 < w ? s_c[(w0 << 6) + 63][i] : c[i];
    for (int x = w0 + 1; x < w; ++x)
#pragma unroll
      for (int i = 0; i < NV; ++i) tot[i] += s_c[(x << 6) + 63][i];
    if (w0 < w)
#pragma unroll
      for (int i = 0; i < NV; ++i) tot[i] += c[i];
#pragma unroll
    for (int i = 0; i < NV; ++i) s_acc[jl][i] += tot[i];
  }
  __syncthreads();
}

// Reduce-scatter of M values over the 64 lanes of a wavefront by recursive
// halving: at each of the six steps a lane keeps one half of its vector (by one
// bit of its lane index), adds its partner's copy of that half and sends the
// other half, so 36 values cost 38 shuffles instead of 36 x 6.  On return lane l
// holds the wave sum of value `idx` (idx >= M: a padding slot, nothing to write).
// Odd lengths are padded with a zero; len tracks how many of a lane's current
// slots are real values.
template <class T, int M, int O>
struct RedScatter {
  static __device__ inline void run(T *a, int lane, int &idx, int &len) {
    constexpr int H = (M + 1) / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const T lo = a[i];
      const T hi = (i + H < M) ? a[i + H] : T(0);
      const T send = up ? lo : hi;
      a[i] = (up ? hi : lo) + __shfl_xor(send, O, 64);
    }
    if (up) {
      idx += H;
      len -= H;
    } else {
      len = min(len, H);
    }
    RedScatter<T, H, O / 2>::run(a, lane, idx, len);
  }
};
template <class T, int M>
struct RedScatter<T, M, 0> {
  static __device__ inline void run(T *, int, int &, int &) {}
};
template <class T, int M>
__device__ inline T wave_reduce_scatter(T (&a)[M], int lane, int &idx) {
  idx = 0;
  int len = M;
  RedScatter<T, M, 32>::run(a, lane, idx, len);
  if (len <= 0) idx = 1 << 30;
  return a[0];
}

// Sum of one value per thread over a 256-thread block, fixed order.
template <class T>
__device__ inline T block_sum256(T v, T *scratch4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) scratch4[w] = v;
  __syncthreads();
  T s = scratch4[0] + scratch4[1] + scratch4[2] + scratch4[3];
  __syncthreads();
  return s;
}

// Sum of one value per thread over a block of NW wavefronts, fixed order.
template <int NW, class T>
__device__ inline T block_sum_w(T v, T *scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  T s = scratch[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s += scratch[i];
  __syncthreads();
  return s;
}

// Sum of n doubles by a 256-thread block in a fixed order (result in every thread).
__device__ inline double block_sum_array(const double *a, int n, double *scratch4) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += a[i];
  return block_sum256(v, scratch4);
}

// Sums of three double arrays of length n in one pass (fixed order; a NULL
// array sums to 0).  Result in every thread.
__device__ inline void block_sum3(const double *a, const double *b, const double *c, int n,
                                  double *scratch12, double out[3]) {
  double va = 0.0, vb = 0.0, vc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    if (a) va += a[i];
    if (b) vb += b[i];
    if (c) vc += c[i];
  }
  va = wave_sum(va);
  vb = wave_sum(vb);
  vc = wave_sum(vc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    scratch12[w] = va;
    scratch12[4 + w] = vb;
    scratch12[8 + w] = vc;
  }
  __syncthreads();
  for (int k = 0; k < 3; ++k)
    out[k] = scratch12[4 * k] + scratch12[4 * k + 1] + scratch12[4 * k + 2] + scratch12[4 * k + 3];
  __syncthreads();
}

template <class T>
__device__ inline T huber_w(T s, T delta) {
  if (delta <= T(0) || s <= delta * delta) return T(1);
  return delta / sqrt(s);
}
template <class T>
__device__ inline T huber_rho(T s, T delta) {
  if (delta <= T(0) || s <= delta * delta) return s;
  return T(2) * delta * sqrt(s) - delta * delta;
}

// World -> camera transform in FP64 from the FP64 state.
template <class PP, class XP>  // pointers to double, generic or global
__device__ inline void transform(PP pose, XP X, double &x, double &y, double &z) {
  x = pose[0] * X[0] + pose[1] * X[1] + pose[2] * X[2] + pose[9];
  y = pose[3] * X[0] + pose[4] * X[1] + pose[5] * X[2] + pose[10];
  z = pose[6] * X[0] + pose[7] * X[1] + pose[8] * X[2] + pose[11];
}

// Residual of one observation in compute type T.  Returns false when the
// point is at or behind the depth threshold (observation masked).
template <class T, class KP>  // KP: pointer to T, generic or global
__device__ inline bool residual(KP K, T x, T y, T z, T uo, T vo, T &r0, T &r1) {
  if (!(z > T(kZMin))) {
    r0 = r1 = T(0);
    return false;
  }
  const T iz = T(1) / z;
  r0 = K[0] * x * iz + K[2] - uo;
  r1 = K[1] * y * iz + K[3] - vo;
  return true;
}

// Jacobians of the residual for a left increment (rho, phi) of the pose and an
// additive point increment: J_pi = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]],
// J_c = J_pi [I | -[P]x], J_p = J_pi R.
template <class T>
__device__ inline void jacobians(const T *K, const double *pose, T x, T y, T z, T Jc[12],
                                 T Jp[6]) {
  const T iz = T(1) / z;
  const T a = K[0] * iz, b = -K[0] * x * iz * iz;
  const T c = K[1] * iz, d = -K[1] * y * iz * iz;
  Jc[0] = a;     Jc[1] = T(0);  Jc[2] = b;
  Jc[3] = b * y; Jc[4] = a * z - b * x; Jc[5] = -a * y;
  Jc[6] = T(0);  Jc[7] = c;     Jc[8] = d;
  Jc[9] = -c * z + d * y; Jc[10] = -d * x; Jc[11] = c * x;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Jp[m] = a * T(pose[m]) + b * T(pose[6 + m]);
    Jp[3 + m] = c * T(pose[3 + m]) + d * T(pose[6 + m]);
  }
}

// se(3) exponential: R = I + A K + B K^2, t = (I + B K + C K^2) rho, K = [phi]x,
// A = sin th / th, B = (1 - cos th) / th^2 = 2 sin^2(th/2) / th^2,
// C = (th - sin th) / th^3, series in th^2 below 1e-4.
__device__ inline void se3_exp(const double xi[6], double R[9], double t[3]) {
  const double p0 = xi[3], p1 = xi[4], p2 = xi[5];
  const double th2 = p0 * p0 + p1 * p1 + p2 * p2;
  double A, B, Cc;
  if (th2 < 1e-8) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    Cc = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    const double th = sqrt(th2);
    const double s = sin(th);
    const double h = sin(0.5 * th) / (0.5 * th);
    A = s / th;
    B = 0.5 * h * h;
    Cc = (th - s) / (th2 * th);
  }
  const double K[9] = {0, -p2, p1, p2, 0, -p0, -p1, p0, 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  double Vm[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    R[i] = I + A * K[i] + B * K2[i];
    Vm[i] = I + B * K[i] + Cc * K2[i];
  }
  for (int i = 0; i < 3; ++i) t[i] = Vm[3 * i] * xi[0] + Vm[3 * i + 1] * xi[1] + Vm[3 * i + 2] * xi[2];
}

// Inverse of a symmetric 3x3 (upper triangle u = [00 01 02 11 12 22]) in FP64.
__device__ inline void inv_sym3(const double u[6], double o[6]) {
  const double a = u[0], b = u[1], c = u[2], d = u[3], e = u[4], f = u[5];
  const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
  const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
  const double det = a * c00 + b * c01 + c * c02;
  const double id = 1.0 / det;
  o[0] = c00 * id; o[1] = c01 * id; o[2] = c02 * id;
  o[3] = c11 * id; o[4] = c12 * id; o[5] = c22 * id;
}

// Inverse of a symmetric positive definite 6x6 in FP64 by Cholesky (A = L L^T,
// A^-1 = L^-T L^-1).  Falls back to the inverse diagonal if A is not
// numerically positive definite.
__device__ inline void inv_spd6(const double A[36], double out[36]) {
  double L[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) L[i] = 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6 && ok; ++j) {
    double s = A[6 * j + j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
    if (!(s > 0.0)) {
      ok = false;
      break;
    }
    const double ljj = sqrt(s);
    L[6 * j + j] = ljj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double t = A[6 * i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = t / ljj;
    }
  }
  if (!ok) {
#pragma unroll
    for (int i = 0; i < 36; ++i) out[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) out[7 * i] = A[7 * i] > 0.0 ? 1.0 / A[7 * i] : 0.0;
    return;
  }
  double Li[36];  // L^-1, lower triangular
#pragma unroll
  for (int i = 0; i < 36; ++i) Li[i] = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    Li[6 * j + j] = 1.0 / L[6 * j + j];
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) s -= L[6 * i + k] * Li[6 * k + j];
      Li[6 * i + j] = s / L[6 * i + i];
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = (i > j ? i : j); k < 6; ++k) s += Li[6 * k + i] * Li[6 * k + j];
      out[6 * i + j] = s;
    }
}

__device__ inline bool lm_active(const LMState *st) { return st->iter < st->max_iters && !st->halted; }

// ------------------------------------------------------------------ linearize
// Point tile: points [j0, j1) and their observations [k0, k1) (contiguous, since
// observations are ordered by point).  Observations are processed 256 at a
// time, one per thread; per-point sums are formed by the first thread of each
// point's run inside the chunk, reading the chunk's contributions from LDS in
// order, so the result does not depend on scheduling.
template <class T, class S>
__global__ __launch_bounds__(kObsChunk) void k_linearize(const ProbDev *__restrict__ probs,
                                                   const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st) || !st->relin) return;
  const int cur = st->cur;
  const T delta = T(st->huber_delta);
  const int j0 = tl.idx * pd.pt_tile;
  const int j1 = min(pd.P, j0 + pd.pt_tile);
  const int k0 = pd.pt_start[j0], k1 = pd.pt_start[j1];

  __shared__ T s_acc[kPtTile][9];
  __shared__ T s_c[kObsChunk][9];
  __shared__ int s_loc[kObsChunk];
  __shared__ double s_red[kObsChunk / 64];
  for (int i = threadIdx.x; i < kPtTile * 9; i += kObsChunk) (&s_acc[0][0])[i] = T(0);

  const auto Kall = as_global((const T *)pd.K);
  const auto uv = as_global((const T *)pd.obs_uv);
  const auto lin = as_global((LinRec<T, S> *)pd.lin);
  const auto poses = as_global((const double *)pd.pose[cur]);
  const auto Xs = as_global((const double *)pd.X[cur]);
  const auto obs_pt = as_global(pd.obs_pt), obs_cam = as_global(pd.obs_cam), obs_rpos = as_global(pd.obs_rpos);
  const auto obs_act = as_global((const uint8_t *)pd.obs_act);
  double cost = 0.0;
  int masked = 0;
  // the observation's own fields for the next pass are loaded while the current pass
  // is processed
  int nj = 0, ncam = 0, ncpos = -1;
  bool non = false;
  T nu = T(0), nv = T(0);
  auto fetch = [&](int k) {
    if (k < k1) {
      nj = obs_pt[k];
      ncam = obs_cam[k];
      ncpos = obs_rpos[k];
      non = obs_act[k] != 0;
      nu = uv[2 * (size_t)k];
      nv = uv[2 * (size_t)k + 1];
    }
  };
  fetch(k0 + (int)threadIdx.x);
  __syncthreads();

  for (int base = k0; base < k1; base += kObsChunk) {
    const int k = base + threadIdx.x;
    const int j = nj, cam = ncam, cpos = ncpos;
    const bool on = non;
    const T ou = nu, ov = nv;
    fetch(k + kObsChunk);
    T c[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = T(0);
    int jl = -1;
    if (k < k1) {
      jl = j - j0;
      const auto pose = poses + 12 * cam;
      double xd, yd, zd;
      transform(pose, Xs + 3 * j, xd, yd, zd);
      const T x = T(xd), y = T(yd), z = T(zd);
      const auto K = Kall + 4 * cam;
      T r0, r1;
      LinRec<T, S> rec;
      if (on && residual<T>(K, x, y, z, ou, ov, r0, r1)) {
        const T s = r0 * r0 + r1 * r1;
        const T w = huber_w(s, delta);
        const T sw = sqrt(w);
        cost += 0.5 * (double)huber_rho(s, delta);
        const T iz = T(1) / z;
        const T fa = K[0] * iz, fb = -K[0] * x * iz * iz;
        const T fc = K[1] * iz, fd = -K[1] * y * iz * iz;
        const T raw[7] = {sw * fa, sw * fb, sw * fc, sw * fd, x, y, z};
        T fq[7];  // stored-precision values: V is formed from them so that V, U and W agree
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          rec.f[i] = Codec<S>::enc(raw[i]);
          fq[i] = Codec<S>::dec(rec.f[i]);
        }
        rec.e[0] = sw * r0;
        rec.e[1] = sw * r1;
        T R[9];
        load_rot(pose, R);
        T Jq[6];
        jp_from(fq, R, Jq);
        const T *P0 = Jq, *P1 = Jq + 3;
        c[0] = P0[0] * P0[0] + P1[0] * P1[0];
        c[1] = P0[0] * P0[1] + P1[0] * P1[1];
        c[2] = P0[0] * P0[2] + P1[0] * P1[2];
        c[3] = P0[1] * P0[1] + P1[1] * P1[1];
        c[4] = P0[1] * P0[2] + P1[1] * P1[2];
        c[5] = P0[2] * P0[2] + P1[2] * P1[2];
        // gradient from the unrounded Jacobian: w J_p^T r
        const T fr[4] = {fa, fb, fc, fd};
        T Jp[6];
        jp_from(fr, R, Jp);
#pragma unroll
        for (int m = 0; m < 3; ++m) c[6 + m] = w * (Jp[m] * r0 + Jp[3 + m] * r1);
      } else {
        masked += on;
#pragma unroll
        for (int i = 0; i < 7; ++i) rec.f[i] = Codec<S>::enc(0.0f);
        rec.e[0] = rec.e[1] = T(0);
      }
      if (cpos >= 0) store_rec(lin + cpos, rec);  // records are kept for free cameras only
    }
    seg_add_scan<T, 9>(c, jl, s_acc, s_c, s_loc);
  }
  const auto V = as_global((T *)pd.V);
  const auto gp = as_global((T *)pd.gp);
  const auto Dp = as_global((T *)pd.Dp);
  for (int jl = threadIdx.x; jl < j1 - j0; jl += kObsChunk) {
    const int j = j0 + jl;
#pragma unroll
    for (int i = 0; i < 6; ++i) V[6 * j + i] = s_acc[jl][i];
#pragma unroll
    for (int i = 0; i < 3; ++i) gp[3 * j + i] = s_acc[jl][6 + i];
    const T d[3] = {s_acc[jl][0], s_acc[jl][3], s_acc[jl][5]};
#pragma unroll
    for (int i = 0; i < 3; ++i) Dp[3 * j + i] = T(fmin(fmax((double)d[i], kDMin), kDMax));
  }
  const double tot = block_sum_w<kObsChunk / 64>(cost, s_red);
  const double nm = block_sum_w<kObsChunk / 64>((double)masked, s_red);
  if (threadIdx.x == 0) {
    pd.part_lin_cost[tl.idx] = tot;
    pd.part_masked[tl.idx] = (int32_t)nm;
  }
}

// ------------------------------------------------------------------ point prep
// V*_j = V_j + lambda D_j inverted in FP64; per free observation Q_k = J_p,k V*_j^-1
// (2x3), from which Y_k = W_k V*_j^-1 = J_c,k^T Q_k is formed where needed.
template <class T, class S>
__global__ __launch_bounds__(256) void k_point_prep(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  const double lam = st->lambda;
  const int j0 = tl.idx * pd.pt_tile;
  const int j1 = min(pd.P, j0 + pd.pt_tile);
  __shared__ T s_vi[kPtTile][6];
  const T *V = (const T *)pd.V;
  const T *Dp = (const T *)pd.Dp;
  T *Vinv = (T *)pd.Vinv;
  for (int jl = threadIdx.x; jl < j1 - j0; jl += 256) {
    const int j = j0 + jl;
    double u[6], o[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) u[i] = (double)V[6 * j + i];
    u[0] += lam * (double)Dp[3 * j + 0];
    u[3] += lam * (double)Dp[3 * j + 1];
    u[5] += lam * (double)Dp[3 * j + 2];
    inv_sym3(u, o);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      s_vi[jl][i] = T(o[i]);
      Vinv[6 * j + i] = T(o[i]);
    }
  }
  __syncthreads();
  const int k0 = pd.pt_start[j0], k1 = pd.pt_start[j1];
  const LinRec<T, S> *lin = (const LinRec<T, S> *)pd.lin;
  const double *poses = pd.pose[st->cur];
  T *Q = (T *)pd.Q;
  for (int k = k0 + threadIdx.x; k < k1; k += 256) {
    const int cpos = pd.obs_rpos[k];
    if (cpos < 0) continue;  // fixed camera: no camera block
    const int jl = pd.obs_pt[k] - j0;
    T f[7], R[9], Jp[6];
    decode(lin[cpos], f);
    load_rot(poses + 12 * pd.obs_cam[k], R);
    jp_from(f, R, Jp);
    const T *vi = s_vi[jl];
    const T M[9] = {vi[0], vi[1], vi[2], vi[1], vi[3], vi[4], vi[2], vi[4], vi[5]};
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        Q[6 * (size_t)cpos + 3 * r + m] = Jp[3 * r] * M[m] + Jp[3 * r + 1] * M[3 + m] + Jp[3 * r + 2] * M[6 + m];
  }
}

// ------------------------------------------------------------------ prior terms
// The prior terms of the Sec. 4.3 objective (Eq. abs, Eq. seq) and the edges of a
// pose graph (Sec. 4.2: sequential, loop-closure and extrinsic constraints, all of
// the form T_i T_j^-1 - M_ij) as weighted squared Frobenius norms of 3x4 pose
// differences, in FP64: the nine rotation entries of a pair carry one weight, the
// three translation entries another.  A pose is held as 12 values,
// R row-major then t; so are the 12-value residuals.  For a left increment
// T <- Exp(xi) T, xi = (rho, phi), row q of d[R | t]/d xi is: for q < 9 (entry
// (a, b) of R) 0 for rho and ([e_m]x R)_ab for phi_m; for q >= 9 (t_r) e_r for rho and
// (-[t]x)_rm for phi_m.  A sequential pair (i, j) has A = T_i T_j^-1, which moves as
// Exp(xi_i) A Exp(-xi_j): d/dxi_i is the same rule at A, d/dxi_j has -(R_A [e_m]x)_ab
// for phi_m (q < 9) and -R_A rows for rho (q >= 9).
__device__ inline void hat3(const double v[3], double H[9]) {
  H[0] = 0.0;   H[1] = -v[2]; H[2] = v[1];
  H[3] = v[2];  H[4] = 0.0;   H[5] = -v[0];
  H[6] = -v[1]; H[7] = v[0];  H[8] = 0.0;
}

// Row q of the left-increment Jacobian of [R | t].
__device__ inline void left_inc_row(const double *R, const double *t, int q, double out[6]) {
  for (int m = 0; m < 6; ++m) out[m] = 0.0;
  if (q < 9) {
    const int a = q / 3, b = q % 3;
    for (int m = 0; m < 3; ++m) {
      double e[3] = {0.0, 0.0, 0.0}, H[9];
      e[m] = 1.0;
      hat3(e, H);
      out[3 + m] = H[3 * a] * R[b] + H[3 * a + 1] * R[3 + b] + H[3 * a + 2] * R[6 + b];
    }
  } else {
    const int r = q - 9;
    double H[9];
    hat3(t, H);
    out[r] = 1.0;
    for (int m = 0; m < 3; ++m) out[3 + m] = -H[3 * r + m];
  }
}

// Row q of d A / d xi_j for A = T_i T_j^-1.
__device__ inline void seq_j_row(const double *RA, int q, double out[6]) {
  for (int m = 0; m < 6; ++m) out[m] = 0.0;
  if (q < 9) {
    const int a = q / 3, b = q % 3;
    for (int m = 0; m < 3; ++m) {
      double e[3] = {0.0, 0.0, 0.0}, H[9];
      e[m] = 1.0;
      hat3(e, H);
      out[3 + m] = -(RA[3 * a] * H[b] + RA[3 * a + 1] * H[3 + b] + RA[3 * a + 2] * H[6 + b]);
    }
  } else {
    const int r = q - 9;
    for (int c = 0; c < 3; ++c) out[c] = -RA[3 * r + c];
  }
}

// A = T_i T_j^-1 = [R_i R_j^T | t_i - R_i R_j^T t_j] as 12 values.
__device__ inline void rel_pose(const double *Ti, const double *Tj, double A[12]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      A[3 * a + b] = Ti[3 * a] * Tj[3 * b] + Ti[3 * a + 1] * Tj[3 * b + 1] + Ti[3 * a + 2] * Tj[3 * b + 2];
  for (int r = 0; r < 3; ++r)
    A[9 + r] = Ti[9 + r] - (A[3 * r] * Tj[9] + A[3 * r + 1] * Tj[10] + A[3 * r + 2] * Tj[11]);
}

// 1/2 (lambda_a sum_i e_a + sum_pairs (w_rot |dR|^2 + w_trans |dt|^2)) at the poses P;
// the block's threads split the terms and sum them in a fixed order.
__device__ inline double prior_abs_term(const ProbDev &pd, const double *P, int i) {
  double e = 0.0;
  for (int q = 0; q < 12; ++q) {
    const double d = P[12 * i + q] - pd.pose0[12 * i + q];
    e += d * d;
  }
  return 0.5 * pd.prior_abs * e;
}
__device__ inline double prior_pair_term(const ProbDev &pd, const double *P, int p) {
  const int2 ij = pd.pp_cam[p];
  const double *M = pd.pp_meas + 12 * (size_t)p;
  double A[12];
  rel_pose(P + 12 * ij.x, P + 12 * ij.y, A);
  double er = 0.0, et = 0.0;
  for (int q = 0; q < 9; ++q) er += (A[q] - M[q]) * (A[q] - M[q]);
  for (int q = 9; q < 12; ++q) et += (A[q] - M[q]) * (A[q] - M[q]);
  return 0.5 * (pd.pp_w[2 * p] * er + pd.pp_w[2 * p + 1] * et);
}
__device__ inline double prior_cost(const ProbDev &pd, const double *P, double *s_red) {
  double c = 0.0;
  if (pd.prior_abs > 0.0)
    for (int i = pd.prior_abs_from + (int)threadIdx.x; i < pd.prior_nodes; i += 256) c += prior_abs_term(pd, P, i);
  for (int p = threadIdx.x; p < pd.n_pp; p += 256) c += prior_pair_term(pd, P, p);
  return block_sum256(c, s_red);
}

// The prior cost of a problem in rig_mode 0, spread over its prior tiles (one block
// each): tile q sums the terms 256 q + t, 256 q + t + 256 n, ... (n tiles) of the
// absolute nodes and then of the pairs, each thread in that order, and the block in a
// fixed order; at the trial poses, and at the current poses on the first call (where
// lm_control records the initial cost).  lm_control adds the tiles' sums in order.
__global__ __launch_bounds__(256) void k_prior_cost(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st) || pd.rig_mode != 0) return;
  __shared__ double s_red[4];
  const int nt = pd.n_pri_tiles, q = tl.idx, t = (int)threadIdx.x, step = 256 * nt;
  const double *Pc = pd.pose[st->cur], *Pt = pd.pose[1 - st->cur];
  const bool first = !st->init_done;
  double cc = 0.0, ct = 0.0;
  if (pd.prior_abs > 0.0)
    for (int i = pd.prior_abs_from + 256 * q + t; i < pd.prior_nodes; i += step) {
      if (first) cc += prior_abs_term(pd, Pc, i);
      ct += prior_abs_term(pd, Pt, i);
    }
  for (int p = 256 * q + t; p < pd.n_pp; p += step) {
    if (first) cc += prior_pair_term(pd, Pc, p);
    ct += prior_pair_term(pd, Pt, p);
  }
  cc = block_sum256(cc, s_red);
  ct = block_sum256(ct, s_red);
  if (t == 0) {
    pd.part_prior[q] = cc;
    pd.part_prior[nt + q] = ct;
  }
}

// Linearisation of the priors at the current poses: thread g < Cf forms the U (upper
// 21) and g (6) contributions of free camera g (its absolute term, then its pairs in
// order); thread g < n_pp forms J_i^T W J_j of pair g when both cameras are free, stored
// as the upper block of S (transposed when i comes after j).
template <class T>
__global__ __launch_bounds__(256) void k_prior_lin(const ProbDev *__restrict__ probs,
                                                   const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const double *P = pd.pose[st->cur];
  const int g = 256 * tl.idx + (int)threadIdx.x;
  if (g < pd.Cf) {
    const int cam = pd.free_cam[g];
    double U[21], gv[6];
    for (int i = 0; i < 21; ++i) U[i] = 0.0;
    for (int i = 0; i < 6; ++i) gv[i] = 0.0;
    auto add_rows = [&](double lam_r, double lam_t, const double *r, auto row_of) {
      for (int q = 0; q < 12; ++q) {
        double J[6];
        row_of(q, J);
        const double lam = q < 9 ? lam_r : lam_t;
        int u = 0;
        for (int a = 0; a < 6; ++a) {
          for (int b = a; b < 6; ++b, ++u) U[u] += lam * J[a] * J[b];
          gv[a] += lam * J[a] * r[q];
        }
      }
    };
    const double *Tc = P + 12 * cam;
    if (pd.prior_abs > 0.0 && cam >= pd.prior_abs_from) {
      double r[12];
      for (int q = 0; q < 12; ++q) r[q] = Tc[q] - pd.pose0[12 * cam + q];
      add_rows(pd.prior_abs, pd.prior_abs, r, [&](int q, double J[6]) { left_inc_row(Tc, Tc + 9, q, J); });
    }
    for (int x = pd.cam_pp_start[g]; x < pd.cam_pp_start[g + 1]; ++x) {
      const int pp = pd.cam_pp[x];
      const int2 ij = pd.pp_cam[pp];
      const double *M = pd.pp_meas + 12 * (size_t)pp;
      const double wr = pd.pp_w[2 * pp], wt = pd.pp_w[2 * pp + 1];
      double A[12], r[12];
      rel_pose(P + 12 * ij.x, P + 12 * ij.y, A);
      for (int q = 0; q < 12; ++q) r[q] = A[q] - M[q];
      if (ij.x == cam)
        add_rows(wr, wt, r, [&](int q, double J[6]) { left_inc_row(A, A + 9, q, J); });
      else
        add_rows(wr, wt, r, [&](int q, double J[6]) { seq_j_row(A, q, J); });
    }
    double *o = pd.prior_diag + 27 * (size_t)g;
    for (int i = 0; i < 21; ++i) o[i] = U[i];
    for (int i = 0; i < 6; ++i) o[21 + i] = gv[i];
  }
  if (g < pd.n_pp && pd.pp_up[g] >= 0) {
    const int2 ij = pd.pp_cam[g];
    double A[12];
    rel_pose(P + 12 * ij.x, P + 12 * ij.y, A);
    double off[36];
    for (int i = 0; i < 36; ++i) off[i] = 0.0;
    const double wr = pd.pp_w[2 * g], wt = pd.pp_w[2 * g + 1];
    for (int q = 0; q < 12; ++q) {
      double Ji[6], Jj[6];
      left_inc_row(A, A + 9, q, Ji);
      seq_j_row(A, q, Jj);
      const double lam = q < 9 ? wr : wt;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) off[6 * a + b] += lam * Ji[a] * Jj[b];
    }
    // block (i, j) of S; the upper block is (min, max) in camera order
    const bool flip = ij.x > ij.y;
    double *o = pd.prior_off + 36 * (size_t)g;
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) o[6 * a + b] = flip ? off[6 * b + a] : off[6 * a + b];
  }
}

// The pair blocks J_i^T W J_j (oriented as the upper block) added to S_ab and
// (transposed) S_ba, after the Schur complement has written them.  Every upper block
// carries at most one pair (pairs are distinct), so no two threads touch one block.
template <class T>
__global__ __launch_bounds__(256) void k_prior_apply(const ProbDev *__restrict__ probs,
                                                     const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int g = 256 * tl.idx + (int)threadIdx.x;
  if (g >= pd.n_pp || pd.pp_up[g] < 0) return;
  const int u = pd.pp_up[g];
  const double *off = pd.prior_off + 36 * (size_t)g;
  T *Sv = (T *)pd.S;
  T *Sab = Sv + 36 * (size_t)pd.up_pos[u];
  T *Sba = Sv + 36 * (size_t)pd.up_tpos[u];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      Sab[6 * a + b] = T((double)Sab[6 * a + b] + off[6 * a + b]);
      Sba[6 * b + a] = T((double)Sba[6 * b + a] + off[6 * a + b]);
    }
}

// Row a of the reduced system from its camera sums tot = [U (upper 21), sum Y W^T
// (upper 21), g_c (6), sum Y g_p (6)] and the prior terms: Marquardt damping, the diagonal block of S,
// the right-hand side b = -g_c + sum Y g_p, the FP64 block-Jacobi inverse, and the
// PCG start (x = 0, r = b, z = p = M^-1 b) with this row's partials of b.b and r.z.
template <class T>
__device__ void finish_camera_row(const ProbDev &pd, const LMState *st, int a, const double tot_in[54]) {
  // the composed-camera view of a rig problem forms its blocks undamped (the rig view
  // damps the rig unknowns) and keeps U for the rig's Marquardt diagonal
  const double lam = pd.rig_mode == 1 ? 0.0 : st->lambda;
  if (pd.rig_mode == 1)
    for (int i = 0; i < 21; ++i) pd.Ucam[21 * (size_t)a + i] = tot_in[i];
  // the prior terms add to U and g_c (their contributions, formed by k_prior_lin)
  double tot[54];
#pragma unroll
  for (int i = 0; i < 54; ++i) tot[i] = tot_in[i];
  if (pd.prior_on) {
    const double *pr = pd.prior_diag + 27 * (size_t)a;
    for (int i = 0; i < 21; ++i) tot[i] += pr[i];
    for (int i = 0; i < 6; ++i) tot[42 + i] += pr[21 + i];
  }
  double Sfull[36], Dc[6];
  int u = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c, ++u) {
      const double Uv = (double)T(tot[u]);
      const double Mv = (double)T(tot[21 + u]);
      const double sv = Uv - Mv;
      Sfull[6 * r + c] = sv;
      Sfull[6 * c + r] = sv;
      if (r == c) Dc[r] = fmin(fmax(Uv, kDMin), kDMax);
    }
#pragma unroll
  for (int r = 0; r < 6; ++r) Sfull[7 * r] += lam * (double)T(Dc[r]);
  T *Sblk = (T *)pd.S + 36 * (size_t)pd.diag_pos[a];
  double Sd[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) {
    Sblk[i] = T(Sfull[i]);
    Sd[i] = (double)T(Sfull[i]);  // the preconditioner inverts the stored block
  }
  double Mi[36];
  inv_spd6(Sd, Mi);
  double *Minv = pd.Minv + 36 * (size_t)a;
#pragma unroll
  for (int i = 0; i < 36; ++i) Minv[i] = Mi[i];
  T *gc = (T *)pd.gc + 6 * a;
  T *Dcv = (T *)pd.Dc + 6 * a;
  T *bv = (T *)pd.brhs + 6 * a;
  T *x = (T *)pd.x + 6 * a;
  T *r = (T *)pd.r + 6 * a;
  T *z = (T *)pd.z + 6 * a;
  T *p = (T *)pd.p0 + 6 * a;
  double bb = 0.0, rz = 0.0;
  double bvals[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T g = T(tot[42 + i]);
    const T b = T(-(double)g + (double)T(tot[48 + i]));
    gc[i] = g;
    Dcv[i] = T(Dc[i]);
    bv[i] = b;
    x[i] = T(0);
    r[i] = b;
    bvals[i] = (double)b;
    bb += bvals[i] * bvals[i];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double zi = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) zi += Mi[6 * i + m] * bvals[m];
    const T zt = T(zi);
    z[i] = zt;
    p[i] = zt;
    rz += bvals[i] * (double)zt;
  }
  pd.part_rz0[a] = rz;
  pd.part_bb[a] = bb;
}

// ------------------------------------------------------------------ Schur: diagonal
// One workgroup per free camera.  Accumulates, over the camera's observations,
// U (upper 21), sum Y W^T = sum J_c^T (Q J_p^T) J_c (upper 21), g_c (6) and
// sum Y g_p = sum J_c^T (Q g_p) (6); then damping,
// the diagonal block of S, the right-hand side, the FP64 block-Jacobi inverse
// and the PCG initial vectors of this row.
template <class T, class S>
__global__ __launch_bounds__(256) void k_schur_diag(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int a = tl.idx;
  const int o0 = pd.cam_obs_start[a], o1 = pd.cam_obs_start[a + 1];
  const LinRec<T, S> *lin = (const LinRec<T, S> *)pd.lin;
  const T *Qall = (const T *)pd.Q;
  const T *gp = (const T *)pd.gp;
  constexpr bool k16 = sizeof(S) == 2;

  T acc[54];
#pragma unroll
  for (int i = 0; i < 54; ++i) acc[i] = T(0);
  // 16-bit storage: the gradient is formed from FP32 Jacobians recomputed here
  int cam = -1;
  const double *pose = nullptr;
  const T *K = nullptr;
  const T delta = T(st->huber_delta);
  if (k16) {
    cam = pd.free_cam[a];
    pose = pd.pose[st->cur] + 12 * cam;
    K = (const T *)pd.K + 4 * cam;
  }
  T Ra[9];
  load_rot(pd.pose[st->cur] + 12 * pd.free_cam[a], Ra);
  for (int o = o0 + threadIdx.x; o < o1; o += 256) {
    const int k = pd.cam_obs[o];
    const int j = pd.obs_pt[k];
    const LinRec<T, S> rec = lin[o];
    T f[7], Jc[12], Jp[6], q[6];
    decode(rec, f);
    jc_from(f, Jc);
    jp_from(f, Ra, Jp);
    const T *Jc0 = Jc, *Jc1 = Jc + 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) q[i] = Qall[6 * (size_t)o + i];
    // M = Q J_p^T (2x2); Y W^T = J_c^T M J_c
    const T m00 = q[0] * Jp[0] + q[1] * Jp[1] + q[2] * Jp[2];
    const T m01 = q[0] * Jp[3] + q[1] * Jp[4] + q[2] * Jp[5];
    const T m10 = q[3] * Jp[0] + q[4] * Jp[1] + q[5] * Jp[2];
    const T m11 = q[3] * Jp[3] + q[4] * Jp[4] + q[5] * Jp[5];
    T Z0[6], Z1[6];
    jct_m(Jc, m00, m01, m10, m11, Z0, Z1);
    acc_jtj_upper(acc, Jc);
    acc_zj_upper(acc + 21, Z0, Z1, Jc);
    T e0 = rec.e[0], e1 = rec.e[1];
    T G0[6], G1[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      G0[r] = Jc0[r];
      G1[r] = Jc1[r];
    }
    if (k16) {
      const double *Xj = pd.X[st->cur] + 3 * j;
      double xd, yd, zd;
      transform(pose, Xj, xd, yd, zd);
      const T x = T(xd), yy = T(yd), z = T(zd);
      const T *uv = (const T *)pd.obs_uv + 2 * (size_t)k;
      T r0, r1;
      if (pd.obs_act[k] && residual<T>(K, x, yy, z, uv[0], uv[1], r0, r1)) {
        const T s = r0 * r0 + r1 * r1;
        const T sw = sqrt(huber_w(s, delta));
        T Jc[12], Jp[6];
        jacobians<T>(K, pose, x, yy, z, Jc, Jp);
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          G0[r] = sw * Jc[r];
          G1[r] = sw * Jc[6 + r];
        }
        e0 = sw * r0;
        e1 = sw * r1;
      } else {
#pragma unroll
        for (int r = 0; r < 6; ++r) G0[r] = G1[r] = T(0);
        e0 = e1 = T(0);
      }
    }
    // Y g_p = J_c^T (Q g_p)
    const T g0 = gp[3 * j], g1 = gp[3 * j + 1], g2 = gp[3 * j + 2];
    const T qg0 = q[0] * g0 + q[1] * g1 + q[2] * g2;
    const T qg1 = q[3] * g0 + q[4] * g1 + q[5] * g2;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      acc[42 + r] += G0[r] * e0 + G1[r] * e1;
      acc[48 + r] += Jc0[r] * qg0 + Jc1[r] * qg1;
    }
  }
  // deterministic block reduction: wave butterflies, then the 4 waves in order
  __shared__ T s_w[4][54];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 54; ++i) {
    const T v = wave_sum(acc[i]);
    if (lane == 0) s_w[w][i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[54];
    for (int i = 0; i < 54; ++i)
      tot[i] = (double)s_w[0][i] + (double)s_w[1][i] + (double)s_w[2][i] + (double)s_w[3][i];
    // NB: the FP32 mode sums its four wave totals in FP64; the sums themselves are FP32.
    finish_camera_row<T>(pd, st, a, tot);
  }
}

// ------------------------------------------------------------------ Schur: off-diagonal
// One wavefront per upper block (a, b): S_ab = -sum_j Y_aj W_bj^T over the
// block's pair list.  With Y = J_c,a^T Q_a and W_b^T = J_p,b^T J_c,b a pair costs
// M = Q_a J_p,b^T (2x2), Z = J_c,a^T M (6x2) and Z J_c,b (6x6); each side's
// Jacobians come from its compact record (camera b's rotation is shared by the
// whole block).  Lanes stride over pairs; one butterfly reduction per block.
template <class T, class S>
__global__ __launch_bounds__(256) void k_schur_off(const ProbDev *__restrict__ probs,
                                                   const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int u = tl.idx * kOffWaves + w;
  if (u >= pd.n_up) return;  // wave-uniform; no block-wide barrier follows
  const int p0 = pd.up_pair_start[u], p1 = pd.up_pair_start[u + 1];
  const LinRec<T, S> *lin = (const LinRec<T, S> *)pd.lin;
  const T *Qall = (const T *)pd.Q;
  T Rb[9];
  load_rot(pd.pose[st->cur] + 12 * pd.free_cam[pd.S_col[pd.up_pos[u]]], Rb);
  T acc[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) acc[i] = T(0);
  for (int p = p0 + lane; p < p1; p += 64) {
    const int2 kk = pd.pairs[p];
    T fa[7], fb[7], Jca[12], Jcb[12], Jpb[6], q[6];
    decode(lin[kk.x], fa);
    decode(lin[kk.y], fb);
#pragma unroll
    for (int i = 0; i < 6; ++i) q[i] = Qall[6 * (size_t)kk.x + i];
    jc_from(fa, Jca);
    jc_from(fb, Jcb);
    jp_from(fb, Rb, Jpb);
    const T m00 = q[0] * Jpb[0] + q[1] * Jpb[1] + q[2] * Jpb[2];
    const T m01 = q[0] * Jpb[3] + q[1] * Jpb[4] + q[2] * Jpb[5];
    const T m10 = q[3] * Jpb[0] + q[4] * Jpb[1] + q[5] * Jpb[2];
    const T m11 = q[3] * Jpb[3] + q[4] * Jpb[4] + q[5] * Jpb[5];
    T z0[6], z1[6];
    jct_m(Jca, m00, m01, m10, m11, z0, z1);
    acc_zj(acc, z0, z1, Jcb);
  }
  // butterfly: every lane ends with all 36 sums; lane e keeps entry e
  T mine = T(0);
#pragma unroll
  for (int i = 0; i < 36; ++i) {
    const T v = wave_sum(acc[i]);
    mine = (lane == i) ? v : mine;
  }
  if (lane < 36) {
    const int r = lane / 6, c = lane % 6;
    T *Sv = (T *)pd.S;
    Sv[36 * (size_t)pd.up_pos[u] + lane] = -mine;
    Sv[36 * (size_t)pd.up_tpos[u] + 6 * c + r] = -mine;
  }
}

// ------------------------------------------------------------------ Schur: point chunks
// Chunk form.  One 1024-thread workgroup per chunk of consecutive points:
//   a. V*_j = V_j + lambda D_j inverted in FP64 for the chunk's points;
//   b. for each of the chunk's records: decoded J_pi and P_c, Q = J_p V*^-1
//      (2x3), Q g_p (2) and the weighted residual, all staged in LDS;
//   c. each entry (a run of at most kChSubItems items of one S block, in point
//      order) is summed by one thread and written as its own partial.
// A block's partials are then summed in chunk order by k_schur_reduce, so S does
// not depend on scheduling and each record is read from HBM once per iteration.
// FP64 runs 512 threads so that the accumulators fit in registers.
template <class T>
constexpr int chunk_threads() { return sizeof(T) == 8 ? kChThreads / 2 : kChThreads; }

// Rows of 8 values in LDS, kept as two arrays of 4-value halves (row l's halves at
// p = base + 4 l and p + hs, hs = 4 x the row capacity) and moved with 16-byte accesses:
// 16 lanes reading or writing consecutive rows then cover the 64 banks once, where whole
// 32-byte rows put two lanes on each bank group, and rows taken in any order spread over
// 16 bank groups instead of 8.
__device__ inline void load8(const float *p, int hs, float o[8]) {
  const float4 a = *(const float4 *)p, b = *(const float4 *)(p + hs);
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
  o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}
__device__ inline void load8(const double *p, int hs, double o[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 a = *(const double2 *)((i < 2 ? p : p + hs) + 2 * (i & 1));
    o[2 * i] = a.x;
    o[2 * i + 1] = a.y;
  }
}
__device__ inline void store8(float *p, int hs, const float v[8]) {
  *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
  *(float4 *)(p + hs) = make_float4(v[4], v[5], v[6], v[7]);
}
__device__ inline void store8(double *p, int hs, const double v[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    *(double2 *)((i < 2 ? p : p + hs) + 2 * (i & 1)) = make_double2(v[2 * i], v[2 * i + 1]);
}

template <class T>
__device__ inline void pair_accumulate(T acc[36], const T *fa_lds, const T *q_lds, const T *fb_lds, int hs,
                                       const T *Rb) {
  T fa[8], q[8], fb[8];
  load8(fa_lds, hs, fa);
  load8(q_lds, hs, q);
  load8(fb_lds, hs, fb);
  T Jca[12], Jcb[12], Jpb[6];
  jc_from(fa, Jca);
  jc_from(fb, Jcb);
  jp_from(fb, Rb, Jpb);
  const T m00 = q[0] * Jpb[0] + q[1] * Jpb[1] + q[2] * Jpb[2];
  const T m01 = q[0] * Jpb[3] + q[1] * Jpb[4] + q[2] * Jpb[5];
  const T m10 = q[3] * Jpb[0] + q[4] * Jpb[1] + q[5] * Jpb[2];
  const T m11 = q[3] * Jpb[3] + q[4] * Jpb[4] + q[5] * Jpb[5];
  T z0[6], z1[6];
  jct_m(Jca, m00, m01, m10, m11, z0, z1);
  acc_zj(acc, z0, z1, Jcb);
}

template <class T, class S>
__global__ __launch_bounds__(chunk_threads<T>()) void k_schur_chunk(const ProbDev *__restrict__ probs,
                                                            const Tile *__restrict__ tiles) {
  constexpr bool k16 = sizeof(S) == 2;
  // chunk_obs_cap / chunk_pts_cap / chunk_cam_cap of the precision mode
  constexpr int cap = sizeof(T) == 8 ? 1024 : k16 ? 1600 : 1984;
  constexpr int pcap = sizeof(T) == 8 ? kChPts / 2 : kChPts;
  constexpr int ccap = sizeof(T) == 8 ? 128 : 256;
  constexpr int nth = chunk_threads<T>();
  extern __shared__ __align__(16) double s_dyn[];
  // per record two rows of 8 (16-byte aligned, read with vector loads):
  // fe = f[0..6], e[0]; qq = Q[0..5], Q g_p[0..1]
  T *s_vi = (T *)s_dyn;           // [pcap][6]
  T *s_fe = s_vi + 6 * pcap;      // [2][cap][4]: rows of 8 in halves
  T *s_qq = s_fe + 8 * cap;       // [2][cap][4]
  constexpr int hs = 4 * cap;     // offset of a row's second half
  T *s_e1 = s_qq + 8 * cap;       // [cap] e[1]; 16-bit storage: [cap][6] FP32 gradient terms
  T *s_R = s_e1 + (k16 ? 6 : 1) * cap;  // [ccap][9] rotations of the chunk's cameras
  int *s_cam = (int *)(s_R + 9 * ccap);  // [ccap]
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int c = tl.idx;
  const int j0 = pd.ch_pt[c], j1 = pd.ch_pt[c + 1];
  const int f0 = pd.ch_f0[c];
  const double *poses = pd.pose[st->cur];
  // the chunk's first records (two per thread): indices and compact records are
  // loaded before the point inverses, so that their latency overlaps them
  const auto lin = as_global((const LinRec<T, S> *)pd.lin);
  const auto gp = as_global((const T *)pd.gp);
  const int k0 = pd.pt_start[j0], k1 = pd.pt_start[j1];
  int kk[2], rp[2], cam[2], jj[2];
  LinRec<T, S> rec[2];
  auto fetch = [&](int base) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      kk[h] = base + h * nth + (int)threadIdx.x;
      rp[h] = kk[h] < k1 ? as_global(pd.obs_rpos)[kk[h]] : -1;
      cam[h] = kk[h] < k1 ? as_global(pd.obs_cam)[kk[h]] : 0;
      jj[h] = kk[h] < k1 ? as_global(pd.obs_pt)[kk[h]] : j0;
      if (rp[h] >= 0) rec[h] = load_rec(lin + rp[h]);
    }
  };
  fetch(k0);
  // a. point inverses
  {
    const double lam = st->lambda;
    const auto V = as_global((const T *)pd.V);
    const auto Dp = as_global((const T *)pd.Dp);
    const auto Vinv = as_global((T *)pd.Vinv);
    for (int jl = threadIdx.x; jl < j1 - j0; jl += nth) {
      const int j = j0 + jl;
      double u[6], o[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) u[i] = (double)V[6 * j + i];
      u[0] += lam * (double)Dp[3 * j + 0];
      u[3] += lam * (double)Dp[3 * j + 1];
      u[5] += lam * (double)Dp[3 * j + 2];
      inv_sym3(u, o);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        s_vi[6 * jl + i] = T(o[i]);
        Vinv[6 * j + i] = T(o[i]);
      }
    }
  }
  // b. rotations of the chunk's cameras (independent of a, before its barrier)
  {
    const int q0 = pd.ch_cam_start[c], nq = pd.ch_cam_start[c + 1] - q0;
    for (int x = threadIdx.x; x < nq; x += nth) {
      const int cm = pd.ch_cam[q0 + x];
      T R[9];
      load_rot(poses + 12 * cm, R);
#pragma unroll
      for (int i = 0; i < 9; ++i) s_R[9 * x + i] = R[i];
      s_cam[x] = cm;
    }
  }
  __syncthreads();
  // b. the records into LDS (chunks hold at most two records per thread, so the loop
  // body runs once; the loop keeps larger chunks correct)
  for (int base = k0; base < k1; base += 2 * nth) {
    if (base != k0) fetch(base);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (rp[h] < 0) continue;  // past the chunk, or a fixed camera: no record
      const int l = rp[h] - f0;
      const int j = jj[h];
      T f[7], R[9], Jp[6];
      decode(rec[h], f);
      load_rot(poses + 12 * cam[h], R);
      jp_from(f, R, Jp);
      const T *vi = s_vi + 6 * (j - j0);
      const T M[9] = {vi[0], vi[1], vi[2], vi[1], vi[3], vi[4], vi[2], vi[4], vi[5]};
      T q[6];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int m = 0; m < 3; ++m)
          q[3 * r + m] = Jp[3 * r] * M[m] + Jp[3 * r + 1] * M[3 + m] + Jp[3 * r + 2] * M[6 + m];
      const T g0 = gp[3 * j], g1 = gp[3 * j + 1], g2 = gp[3 * j + 2];
      T fe[8], qq[8];
#pragma unroll
      for (int i = 0; i < 7; ++i) fe[i] = f[i];
      fe[7] = rec[h].e[0];
#pragma unroll
      for (int i = 0; i < 6; ++i) qq[i] = q[i];
      qq[6] = q[0] * g0 + q[1] * g1 + q[2] * g2;
      qq[7] = q[3] * g0 + q[4] * g1 + q[5] * g2;
      store8(s_fe + 4 * l, hs, fe);
      store8(s_qq + 4 * l, hs, qq);
      if (k16) {
        // 16-bit storage: this record's gradient term w J_c^T r from FP32 Jacobians
        const int cm = cam[h];
        const double *pose = poses + 12 * cm;
        const T *K = (const T *)pd.K + 4 * cm;
        const T *uv = (const T *)pd.obs_uv + 2 * (size_t)kk[h];
        double xd, yd, zd;
        transform(pose, pd.X[st->cur] + 3 * (size_t)j, xd, yd, zd);
        const T xv = T(xd), yv = T(yd), zv = T(zd);
        T r0, r1, gk[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) gk[r] = T(0);
        if (pd.obs_act[kk[h]] && residual<T>(K, xv, yv, zv, uv[0], uv[1], r0, r1)) {
          const T w = huber_w(r0 * r0 + r1 * r1, T(st->huber_delta));
          T Jg[12], Jpg[6];
          jacobians<T>(K, pose, xv, yv, zv, Jg, Jpg);
#pragma unroll
          for (int r = 0; r < 6; ++r) gk[r] = w * (Jg[r] * r0 + Jg[6 + r] * r1);
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) s_e1[6 * l + r] = gk[r];
      } else {
        s_e1[l] = rec[h].e[1];
      }
    }
  }
  __syncthreads();
  // c. entries, one thread each: sums over at most kChSubItems items of one
  // block, all item indices loaded before the arithmetic (item h of the 64 entries of
  // a wavefront is one contiguous run: one coalesced load)
  const int e0 = pd.ch_ent[c], e1 = pd.ch_ent[c + 1];
  const auto pdg = as_global((T *)pd.part_d);
  const auto pof = as_global((T *)pd.part_o);
  const auto items_g = as_global(pd.ent_items);
  for (int e = e0 + threadIdx.x; e < e1; e += nth) {
    const int tgt = as_global(pd.ent_tgt)[e];
    const int i0 = as_global(pd.ent_start)[e], n = as_global(pd.ent_len)[e];
    const int slot = as_global(pd.ent_slot)[e];
    const int lc = as_global(pd.ent_cam)[e];
    const T *R = s_R + 9 * lc;
    uint32_t items[kChSubItems];
#pragma unroll
    for (int h = 0; h < kChSubItems; ++h) items[h] = h < n ? items_g[i0 + kEntSlice * h] : 0u;
    if (tgt < pd.Cf) {
      // diagonal block of camera cam over its observations, in two passes to bound
      // the live accumulators: U, g_c, Y g_p (33), then Y W^T (21)
      const auto o = pdg + 54 * (size_t)slot;
      T acc[33];
#pragma unroll
      for (int i = 0; i < 33; ++i) acc[i] = T(0);
#pragma unroll
      for (int h = 0; h < kChSubItems; ++h) {
        if (h >= n) break;
        const int l = (int)items[h];
        T fe[8], qq[8];
        load8(s_fe + 4 * l, hs, fe);
        load8(s_qq + 4 * l, hs, qq);
        T Jc[12];
        jc_from(fe, Jc);
        const T *Jc0 = Jc, *Jc1 = Jc + 6;
        acc_jtj_upper(acc, Jc);
#pragma unroll
        for (int r = 0; r < 6; ++r) acc[27 + r] += Jc0[r] * qq[6] + Jc1[r] * qq[7];
        if (k16) {
#pragma unroll
          for (int r = 0; r < 6; ++r) acc[21 + r] += s_e1[6 * l + r];
        } else {
          const T e0v = fe[7], e1v = s_e1[l];
#pragma unroll
          for (int r = 0; r < 6; ++r) acc[21 + r] += Jc0[r] * e0v + Jc1[r] * e1v;
        }
      }
      // partial layout: U (21), Y W^T (21), g_c (6), Y g_p (6)
#pragma unroll
      for (int i = 0; i < 21; ++i) o[i] = acc[i];
#pragma unroll
      for (int i = 21; i < 33; ++i) o[21 + i] = acc[i];
      T acw[21];
#pragma unroll
      for (int i = 0; i < 21; ++i) acw[i] = T(0);
#pragma unroll
      for (int h = 0; h < kChSubItems; ++h) {
        if (h >= n) break;
        const int l = (int)items[h];
        T f[8], q[8];
        load8(s_fe + 4 * l, hs, f);
        load8(s_qq + 4 * l, hs, q);
        T Jc[12], Jp[6];
        jc_from(f, Jc);
        jp_from(f, R, Jp);
        const T m00 = q[0] * Jp[0] + q[1] * Jp[1] + q[2] * Jp[2];
        const T m01 = q[0] * Jp[3] + q[1] * Jp[4] + q[2] * Jp[5];
        const T m10 = q[3] * Jp[0] + q[4] * Jp[1] + q[5] * Jp[2];
        const T m11 = q[3] * Jp[3] + q[4] * Jp[4] + q[5] * Jp[5];
        T z0[6], z1[6];
        jct_m(Jc, m00, m01, m10, m11, z0, z1);
        acc_zj_upper(acw, z0, z1, Jc);
      }
#pragma unroll
      for (int i = 0; i < 21; ++i) o[21 + i] = acw[i];
    } else {
      T acc[36];
#pragma unroll
      for (int i = 0; i < 36; ++i) acc[i] = T(0);
#pragma unroll
      for (int h = 0; h < kChSubItems; ++h) {
        if (h >= n) break;
        const int p = (int)(items[h] & 0xffffu), qq = (int)(items[h] >> 16);
        pair_accumulate<T>(acc, s_fe + 4 * p, s_qq + 4 * p, s_fe + 4 * qq, hs, R);
      }
      const auto o = pof + 36 * (size_t)slot;
#pragma unroll
      for (int i = 0; i < 36; ++i) o[i] = acc[i];
    }
  }
}

// Upper blocks, one wave each (four per workgroup).  The block's chunk partials are
// contiguous rows of 36 T in chunk order; each lane loads 16 bytes (V elements) of a
// row, so one wave instruction reads RW whole rows (7 in FP32, 3 in FP64) contiguously.
// Lane (row slot r, quad q) sums rows r, r + RW, r + 2 RW, ... in FP64 in that order; the
// RW slot sums are then added in slot order, and the element is written as S_ab = -sum
// and into S_ba, its transpose.
template <class T>
__global__ __launch_bounds__(256) void k_schur_reduce(const ProbDev *__restrict__ probs,
                                                      const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte load
  constexpr int Q = 36 / V;               // loads per row
  constexpr int RW = 64 / Q;              // rows per wave instruction
  using Vec = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  const int lane = threadIdx.x & 63;
  const int u = 4 * tl.idx + (threadIdx.x >> 6);
  if (u >= pd.n_up) return;  // whole waves: no workgroup barrier follows
  const int r = lane / Q, q = lane - Q * (lane / Q);
  const bool act = r < RW;
  const int b0 = pd.blk_start[pd.Cf + u], n = pd.blk_start[pd.Cf + u + 1] - b0;
  const T *part = (const T *)pd.part_o + 36 * (size_t)(b0 - pd.n_dent) + V * q;
  double acc[V];
#pragma unroll
  for (int k = 0; k < V; ++k) acc[k] = 0.0;
  for (int x0 = r; x0 < n; x0 += 4 * RW) {  // four rows per lane in flight, summed in order
    Vec v[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int x = x0 + h * RW;
      v[h] = (act && x < n) ? *(const Vec *)(part + 36 * (size_t)x) : Vec{};
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const T *e = (const T *)&v[h];
#pragma unroll
      for (int k = 0; k < V; ++k) acc[k] += (double)e[k];
    }
  }
  double tot[V];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    tot[k] = 0.0;
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) tot[k] += __shfl(acc[k], rr * Q + q, 64);
  }
  if (lane < Q) {
    T *Sv = (T *)pd.S;
    const size_t pu = 36 * (size_t)pd.up_pos[u], pt = 36 * (size_t)pd.up_tpos[u];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int e = V * q + k, rr = e / 6, cc = e - 6 * (e / 6);
      const T val = T(-tot[k]);
      Sv[pu + e] = val;
      Sv[pt + 6 * cc + rr] = val;
    }
  }
}

// Camera rows, one 1024-thread workgroup each: wave w sums the w-th of 16
// consecutive segments of the row's diagonal partials (rows of 54) in FP64 and
// the segment sums are added in order into row_tot; k_schur_finish then runs
// finish_camera_row, one thread per camera (kept apart for its registers).
template <class T>
__global__ __launch_bounds__(1024) void k_schur_rows(const ProbDev *__restrict__ probs,
                                                     const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int a = tl.idx;
  const int b0 = pd.blk_start[a], n = pd.blk_start[a + 1] - b0;
  const int q = (n + 15) / 16, x0 = wv * q, x1 = min(n, x0 + q);
  const T *part = (const T *)pd.part_d + 54 * (size_t)b0;
  __shared__ double s_t[16][54];
  double t = 0.0;
  if (lane < 54)
    for (int x = x0; x < x1; x += 8) {
      T v[8];
#pragma unroll
      for (int h = 0; h < 8; ++h) v[h] = x + h < x1 ? part[54 * (size_t)(x + h) + lane] : T(0);
#pragma unroll
      for (int h = 0; h < 8; ++h) t += (double)v[h];
    }
  if (lane < 54) s_t[wv][lane] = t;
  __syncthreads();
  if (threadIdx.x < 54) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) v += s_t[w][threadIdx.x];
    pd.row_tot[54 * (size_t)a + threadIdx.x] = v;
  }
}

template <class T>
__global__ __launch_bounds__(64) void k_schur_finish(const ProbDev *__restrict__ probs,
                                                     const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int a = 64 * tl.idx + (int)threadIdx.x;
  if (a >= pd.Cf) return;
  double tot[54];
  // no records (a pose graph): the rows kernel does not run and every row sum is zero
  if (pd.Nf > 0) {
    const double *rt = pd.row_tot + 54 * (size_t)a;
#pragma unroll
    for (int i = 0; i < 54; ++i) tot[i] = rt[i];
  } else {
#pragma unroll
    for (int i = 0; i < 54; ++i) tot[i] = 0.0;
  }
  finish_camera_row<T>(pd, st, a, tot);
}

// ------------------------------------------------------------------ PCG
// Tile = pd.pcg_rows (4 or 16) consecutive rows of one problem; in the two-kernel
// form each wave of the 256-thread workgroup takes every fourth row of the tile.
// Iteration it (0-based):
//   spmv(it):   it >= 1: stop if ||r_it|| <= tol ||b||; beta = rz_it / rz_{it-1};
//               p_it = z + beta p_{it-1} (formed on the fly for every column read);
//               q = S p_it; partial p_it . q.
//   update(it): alpha = rz_it / (p.q); x += alpha p; r -= alpha q; z = M^-1 r;
//               partials r.z and r.r.
// A tile reads the problem's PCG flags once, by one thread, and broadcasts them
// through LDS: another tile of the same problem may set them while this one
// runs, and every thread must take the same branch.  (A single launch per
// iteration, with the last workgroup doing the update, measured slower on
// MI355X: the device-scope fences it needs cost more than a kernel boundary;
// so did a cooperative kernel with grid barriers.)

__device__ inline bool pcg_go(const LMState *st, int it, int lim, int *s_flag);
__device__ inline bool pcg_go(const LMState *st, int it, int *s_flag) {
  return pcg_go(st, it, it + 1, s_flag);
}
// go while the problem is active, not done, and lim <= pcg_max
__device__ inline bool pcg_go(const LMState *st, int it, int lim, int *s_flag) {
  if (threadIdx.x == 0) s_flag[0] = (lm_active(st) && !st->pcg_done && lim <= st->pcg_max) ? 1 : 0;
  __syncthreads();
  const bool go = s_flag[0] != 0;
  __syncthreads();
  return go;
}

template <class T>
__device__ void pcg_spmv_tile(const ProbDev *__restrict__ probs, const Tile tl, int it) {
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  __shared__ int s_flag[1];
  __shared__ double s_red[4];
  __shared__ double s_pq[4];
  if (!pcg_go(st, it, s_flag)) return;
  double beta = 0.0;
  if (it == 0) {
    // tile 0 alone sums ||b||^2 and r.z over the cameras (the next launch reads them);
    // with b = 0 the other tiles' products are zero and harmless
    if (tl.idx == 0) {
      const double bb = block_sum_array(pd.part_bb, pd.Cf, s_red);
      const double rz0 = block_sum_array(pd.part_rz0, pd.Cf, s_red);
      if (threadIdx.x == 0) {
        st->pcg_bb = bb;
        st->pcg_rz0 = rz0;
      }
      if (!(bb > 0.0)) {
        if (threadIdx.x == 0) {
          st->pcg_done = 1;
          st->pcg_iters = 0;
        }
        return;
      }
    }
  } else {
    __shared__ double s_red3[12];
    double sums[3];  // r.r, rz_it, rz_{it-1}
    block_sum3(pd.part_rr, pd.part_rz[it & 1], it == 1 ? nullptr : pd.part_rz[(it - 1) & 1],
               pd.n_pcg_tiles, s_red3, sums);
    const double bb = st->pcg_bb;
    if (sqrt(sums[0]) <= st->pcg_tol * sqrt(bb)) {
      if (tl.idx == 0 && threadIdx.x == 0) {
        st->pcg_done = 1;
        st->pcg_iters = it;
      }
      return;
    }
    const double rz_old = (it == 1) ? st->pcg_rz0 : sums[2];
    beta = sums[1] / rz_old;
  }
  const T tb = T(beta);
  const T *z = (const T *)pd.z;
  const T *pold = (const T *)((it & 1) ? pd.p0 : pd.p1);  // p_{it-1}
  const T *pin = (const T *)pd.p0;                        // p_0 when it == 0
  T *pout = (T *)((it & 1) ? pd.p1 : pd.p0);              // p_it
  T *q = (T *)pd.q;
  const T *S = (const T *)pd.S;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / 6, i = lane % 6;
  double pq = 0.0;
  for (int rr = w; rr < pd.pcg_rows; rr += 4) {
    const int a = tl.idx * pd.pcg_rows + rr;
    if (a >= pd.Cf) break;
    T acc = T(0);
    if (lane < 60) {
      const int b1 = pd.S_rowptr[a + 1];
#pragma unroll 2
      for (int blk = pd.S_rowptr[a] + g; blk < b1; blk += 10) {
        const int c = pd.S_col[blk];
        const T *Srow = S + 36 * (size_t)blk + 6 * i;
        T sv[6], pc[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) sv[m] = Srow[m];
        if (it == 0) {
#pragma unroll
          for (int m = 0; m < 6; ++m) pc[m] = pin[6 * c + m];
        } else {
#pragma unroll
          for (int m = 0; m < 6; ++m) pc[m] = z[6 * c + m] + tb * pold[6 * c + m];
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) acc += sv[m] * pc[m];
      }
    }
    // lanes 6g + i hold partial sums of output i; gather them in a fixed order
    T qi = T(0);
#pragma unroll
    for (int gg = 0; gg < 10; ++gg) qi += __shfl(acc, 6 * gg + i, 64);
    if (lane < 6) {
      const T pa = (it == 0) ? pin[6 * a + lane] : z[6 * a + lane] + tb * pold[6 * a + lane];
      q[6 * a + lane] = qi;
      if (it > 0) pout[6 * a + lane] = pa;
      pq += (double)pa * (double)qi;
    }
  }
  const double tot = block_sum256(pq, s_pq);
  if (threadIdx.x == 0) pd.part_pq[tl.idx] = tot;
}

template <class T>
__device__ void pcg_update_tile(const ProbDev *__restrict__ probs, const Tile tl, int it) {
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  __shared__ int s_flag[1];
  __shared__ double s_red[4];
  __shared__ double s_red2[4];
  __shared__ T s_r[kPcgRowsMax * 6];
  if (!pcg_go(st, it, s_flag)) return;
  __shared__ double s_red3[12];
  double sums[3];  // p.q, rz_it
  block_sum3(pd.part_pq, it == 0 ? nullptr : pd.part_rz[it & 1], nullptr, pd.n_pcg_tiles, s_red3, sums);
  const double pq = sums[0];
  if (!(pq > 0.0)) {  // breakdown: keep x, stop
    if (tl.idx == 0 && threadIdx.x == 0) {
      st->pcg_done = 1;
      st->pcg_iters = it + 1;
    }
    return;
  }
  const double rz = (it == 0) ? st->pcg_rz0 : sums[1];
  const double alpha = rz / pq;
  const T ta = T(alpha);
  const T *p = (const T *)((it & 1) ? pd.p1 : pd.p0);
  const T *q = (const T *)pd.q;
  T *x = (T *)pd.x;
  T *r = (T *)pd.r;
  T *z = (T *)pd.z;
  const int rbeg = tl.idx * pd.pcg_rows;
  const int rend = min(pd.Cf, rbeg + pd.pcg_rows);
  double rzp = 0.0, rrp = 0.0;
  // one thread per row element (6 * pcg_rows of them)
  const int e = threadIdx.x;
  const int a = rbeg + e / 6;
  if (e < 6 * pd.pcg_rows && a < rend) {
    const size_t idx = 6 * (size_t)a + (e % 6);
    x[idx] = x[idx] + ta * p[idx];
    const T rn = r[idx] - ta * q[idx];
    r[idx] = rn;
    s_r[e] = rn;
  }
  __syncthreads();
  if (e < 6 * pd.pcg_rows && a < rend) {
    const int i = e % 6;
    const double *Mi = pd.Minv + 36 * (size_t)a + 6 * i;
    const T *rr = s_r + 6 * (e / 6);
    double zi = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) zi += Mi[m] * (double)rr[m];
    const T zt = T(zi);
    z[6 * (size_t)a + i] = zt;
    rzp = (double)rr[i] * (double)zt;
    rrp = (double)rr[i] * (double)rr[i];
  }
  const double trz = block_sum256(rzp, s_red);
  const double trr = block_sum256(rrp, s_red2);
  if (threadIdx.x == 0) {
    pd.part_rz[(it + 1) & 1][tl.idx] = trz;
    pd.part_rr[tl.idx] = trr;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_pcg_spmv(const ProbDev *__restrict__ probs,
                                                  const Tile *__restrict__ tiles, int it) {
  pcg_spmv_tile<T>(probs, tiles[blockIdx.x], it);
}

template <class T>
__global__ __launch_bounds__(256) void k_pcg_update(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles, int it) {
  pcg_update_tile<T>(probs, tiles[blockIdx.x], it);
}

// One-reduction form (Chronopoulos & Gear 1989): the same block-Jacobi PCG
// iterates with both inner products of an iteration taken in one reduction, so
// one launch per iteration suffices and a launch reads only the columns its own
// rows touch.  With u = M^-1 r, w = S u, s = S p:
//   gamma_i = r_i.u_i, delta_i = w_i.u_i,
//   beta_i = gamma_i / gamma_{i-1} (beta_0 = 0),
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})   (= gamma_i / p_i.S p_i),
//   p_i = u_i + beta_i p_{i-1}, s_i = w_i + beta_i s_{i-1},
//   x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i,
//   u_{i+1} = M^-1 r_{i+1}, w_{i+1} = S u_{i+1}.
// Launch i sums the tile partials of gamma_i, delta_i and ||r_i||^2 handed in by
// launch i - 1 (fixed order), tests ||r_i|| <= tol ||b||, then forms s_i, r_{i+1}
// and u_{i+1} for every column its rows read (into LDS; each column's owner
// writes them), p_i and x_{i+1} for its rows, w_{i+1} = S u_{i+1} for its rows,
// and its partials of gamma_{i+1}, delta_{i+1} and ||r_{i+1}||^2.  Vectors and
// partials alternate between two buffers by parity; the cg_start launch forms
// w_0 = S u_0 and the first partials.
template <int NW>
__device__ inline void cg_partials(double *part, int n_tiles, int tile, double g, double d, double rr,
                                   double *s3nw) {
  g = wave_sum(g);
  d = wave_sum(d);
  rr = wave_sum(rr);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    s3nw[w] = g;
    s3nw[NW + w] = d;
    s3nw[2 * NW + w] = rr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s3nw[0], b = s3nw[NW], c = s3nw[2 * NW];
#pragma unroll
    for (int k = 1; k < NW; ++k) {
      a += s3nw[k];
      b += s3nw[NW + k];
      c += s3nw[2 * NW + k];
    }
    part[tile] = a;
    part[n_tiles + tile] = b;
    part[2 * n_tiles + tile] = c;
  }
}

// NW waves per tile, wave w taking rows w, w + NW, ...: 4 for 4-row tiles (and mixed
// batches), 16 for tiles of 16 or 32 rows, so that no wave walks more than two rows.
template <class T, int NW>
__global__ __launch_bounds__(64 * NW) void k_cg_start(const ProbDev *__restrict__ probs,
                                                      const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  __shared__ int s_flag[1];
  __shared__ double s_red[3 * NW];
  if (threadIdx.x == 0) pd.cg_flag[tl.idx] = 0u;  // the resident PCG's barrier flags
  if (threadIdx.x == 0) s_flag[0] = lm_active(st) ? 1 : 0;
  __syncthreads();
  if (!s_flag[0]) return;
  // tile 0 alone sums ||b||^2 over the cameras and sets the flags the first step
  // reads (its loads issued here, reduced after its rows); with b = 0 every tile's
  // products are zero and harmless
  double vbb = 0.0;
  if (tl.idx == 0 && threadIdx.x < 256) {
    constexpr int kU = 8;  // a thread's loads of kU strides issued together, summed in order
    const int n = pd.Cf;
    for (int i0 = threadIdx.x; i0 < n; i0 += 256 * kU) {
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = pd.part_bb[min(i0 + 256 * u, n - 1)];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (i0 + 256 * u < n) vbb += v[u];
    }
  }
  const T *u = (const T *)pd.cg_u[0];
  const T *r = (const T *)pd.cg_r[0];
  T *w = (T *)pd.cg_w[0];
  T *sv = (T *)pd.cg_s[0];
  T *p = (T *)pd.p0;
  const T *S = (const T *)pd.S;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane / 6, i = lane % 6;
  double pg = 0.0, pdl = 0.0, prr = 0.0;
  for (int rr = wv; rr < pd.pcg_rows; rr += NW) {
    const int a = tl.idx * pd.pcg_rows + rr;
    if (a >= pd.Cf) break;
    T acc = T(0);
    if (lane < 60) {
      // four blocks at a time, their loads issued before the first product (the sum
      // stays in block order)
      const int b1 = pd.S_rowptr[a + 1];
      int blk = pd.S_rowptr[a] + g;
      for (; blk + 30 < b1; blk += 40) {
        T sv[4][6], uv[4][6];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = pd.S_col[blk + 10 * q];
          const T *Srow = S + 36 * (size_t)(blk + 10 * q) + 6 * i;
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            sv[q][m] = Srow[m];
            uv[q][m] = u[6 * c + m];
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int m = 0; m < 6; ++m) acc += sv[q][m] * uv[q][m];
      }
      for (; blk < b1; blk += 10) {
        const int c = pd.S_col[blk];
        const T *Srow = S + 36 * (size_t)blk + 6 * i;
#pragma unroll
        for (int m = 0; m < 6; ++m) acc += Srow[m] * u[6 * c + m];
      }
    }
    T wi = T(0);
#pragma unroll
    for (int gg = 0; gg < 10; ++gg) wi += __shfl(acc, 6 * gg + i, 64);
    if (lane < 6) {
      const size_t idx = 6 * (size_t)a + lane;
      w[idx] = wi;
      sv[idx] = T(0);  // s_{-1}
      p[idx] = T(0);   // p_{-1}
      const double ui = (double)u[idx], ri = (double)r[idx];
      pg += ri * ui;
      pdl += (double)wi * ui;
      prr += ri * ri;
    }
  }
  cg_partials<NW>(pd.part_cg[0], pd.n_pcg_tiles, tl.idx, pg, pdl, prr, s_red);
  if (tl.idx == 0) {
    // not s_red: thread 0 may still be reading the partials there.  The order of
    // block_sum_array over 256 threads; waves past the fourth add zeros
    __shared__ double s_bb[NW];
    const double bb = block_sum_w<NW>(vbb, s_bb);
    if (threadIdx.x == 0) {
      st->pcg_bb = bb;
      st->pcg_done = (bb > 0.0) ? 0 : 1;
      st->pcg_iters = 0;
    }
  }
}

// One PCG iteration per launch, 1024 threads per tile of pd.pcg_rows rows.  A
// launch is short and its data sit in L2 / the Infinity Cache, so its time is
// set by dependent memory round trips, not bandwidth: every load that does not
// need this iteration's alpha and beta (the S blocks of the tile's rows, the
// previous vectors of every column the tile reads, the M^-1 rows, the partial
// sums and the LM scalars) is issued before the one reduction barrier.
//   column pass: thread (l, m) owns component m of column l (up to 170 columns
//                in registers, the rest in a second sweep);
//   product:     row = 1024 / pcg_rows lanes (4 waves for 4-row tiles, 1 for 16,
//                half a wave for 32) in groups of 6 lanes (10 per wave, 5 per half
//                wave), cg_pre<T>() S blocks per lane held in registers, group sums
//                by a fixed shuffle tree, the waves of a row in order.
constexpr int kCgThreads = 1024;
template <class T>
constexpr int cg_pre() { return sizeof(T) == 4 ? 4 : 1; }  // within 128 VGPRs at 16 waves per CU
constexpr int kCgColThreads = 1020;  // 170 columns x 6 components

template <class T>
__device__ inline void cg_column(int m, T tb, T ta, const T (&w0)[6], const T (&s0)[6], const T (&r0)[6],
                                 const double (&mrow)[6], T &sm, T &rm, T &um) {
  T sn[6], rn[6];
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    sn[n] = w0[n] + tb * s0[n];
    rn[n] = r0[n] - ta * sn[n];
  }
  double z = 0.0;
#pragma unroll
  for (int n = 0; n < 6; ++n) z += mrow[n] * (double)rn[n];
  um = T(z);
  sm = sn[0];
  rm = rn[0];
#pragma unroll
  for (int n = 1; n < 6; ++n)
    if (n == m) {
      sm = sn[n];
      rm = rn[n];
    }
}

// RC: the rows per tile when the launch knows them (4, 16, 32), else 0 (read per problem).
template <class T, int RC>
__device__ __forceinline__ void cg_step_body(const ProbDev &pd, const int tile, int it) {
  extern __shared__ double s_dyn[];
  T *ul = (T *)s_dyn;  // [tile columns][6]: u_{it+1} of every column this tile reads
  __shared__ double s_red[48];
  __shared__ T s_w[kPcgRowsMax][4][6];
  __shared__ T s_ro[kPcgRowsMax][6], s_uo[kPcgRowsMax][6];
  __shared__ double s_fin[12];
  __shared__ int s_flag[1];
  const Tile tl{0, tile};
  const LMState *st = pd.st;
  // A launch that finds the solve finished leaves before issuing any other load: the
  // graph of an LM iteration holds every allowed PCG step, and once the PCG has
  // converged the rest only pass through here.  (A tile that sees the flag its own
  // launch's tile 0 has just set leaves as it would after its own convergence test.)
  if (!(lm_active(st) && !st->pcg_done && it < st->pcg_max)) return;
  const int t = threadIdx.x;
  const int pr = it & 1, cu = (it + 1) & 1;
  const int nt = pd.n_pcg_tiles;
  const int R = RC ? RC : pd.pcg_rows;    // rows per tile: 4, 16 or 32
  const int Lr = kCgThreads / R;          // lanes per row: 256, 64 or 32
  const int wpr = Lr >= 64 ? Lr / 64 : 1;  // waves per row (a half-wave row counts as one)
  const int row0 = tl.idx * R, row1 = min(pd.Cf, row0 + R);
  const int ncmax = pd.max_tcols;
  const int32_t *tcol = pd.tcol + (size_t)tl.idx * ncmax;
  const T *r0 = (const T *)pd.cg_r[pr];
  const T *u0 = (const T *)pd.cg_u[pr];
  const T *w0 = (const T *)pd.cg_w[pr];
  const T *s0 = (const T *)pd.cg_s[pr];
  const T *p0 = (const T *)(pr ? pd.p1 : pd.p0);
  const T *S = (const T *)pd.S;
  T *x = (T *)pd.x;
  // ---- loads that do not depend on this iteration's scalars
  const double tol = st->pcg_tol, bb = st->pcg_bb;
  const double gprev = st->cg_gamma[pr], aprev = st->cg_alpha[pr];
  double pg = 0.0, pdl = 0.0, prr = 0.0;
  {
    const double *part = pd.part_cg[pr];
    for (int k = t; k < nt; k += kCgThreads) {
      pg += part[k];
      pdl += part[nt + k];
      prr += part[2 * nt + k];
    }
  }
  const int l = t / 6, m = t - 6 * (t / 6);
  const int c = (t < kCgColThreads && l < ncmax) ? tcol[l] : -1;
  const bool has_col = c >= 0;
  T cw[6], cs[6], cr[6];
  double mrow[6];
  T u0m = T(0), p0m = T(0), xm = T(0);
  if (has_col) {
    const size_t b = 6 * (size_t)c;
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      cw[n] = w0[b + n];
      cs[n] = s0[b + n];
      cr[n] = r0[b + n];
      mrow[n] = pd.Minv[36 * (size_t)c + 6 * m + n];
    }
  }
  const bool own = has_col && c >= row0 && c < row1;
  if (own) {
    u0m = u0[6 * (size_t)c + m];
    p0m = p0[6 * (size_t)c + m];
    xm = x[6 * (size_t)c + m];
  }
  const int lrs = R == kPcgRows ? 8 : (R == kPcgRowsSparse ? 6 : 5);  // log2(Lr)
  const int lane = t & 63, rw = t >> lrs;
  const int h = t & (Lr - 1);                        // lane within the row
  const int q = Lr >= 64 ? (h >> 6) : 0;             // wave within the row
  const int hs = Lr >= 64 ? (h & 63) : h;            // lane within the row's wave segment
  const int gps = Lr >= 64 ? 10 : 5;                 // groups of 6 lanes per segment
  const int g = hs / 6, i = hs - 6 * (hs / 6);
  const int a = row0 + rw;
  const int bstep = gps * wpr;  // blocks between one lane group's consecutive blocks
  const bool spl = g < gps && a < row1;
  int b0 = 0, b1 = 0;
  if (spl) {
    b0 = pd.S_rowptr[a] + gps * q + g;
    b1 = pd.S_rowptr[a + 1];
  }
  constexpr int kCgPre = cg_pre<T>();
  T sreg[kCgPre][6];
  int lreg[kCgPre];
#pragma unroll
  for (int k = 0; k < kCgPre; ++k) {
    const int blk = b0 + bstep * k;
    lreg[k] = -1;
    if (blk < b1) {
      lreg[k] = pd.S_lcol[blk];
#pragma unroll
      for (int n = 0; n < 6; ++n) sreg[k][n] = S[36 * (size_t)blk + 6 * i + n];
    } else {
#pragma unroll
      for (int n = 0; n < 6; ++n) sreg[k][n] = T(0);
    }
  }
  // ---- the one reduction: gamma_it, delta_it, ||r_it||^2 and the activity flag
  if (t == 0) s_flag[0] = (lm_active(st) && !st->pcg_done && it < st->pcg_max) ? 1 : 0;
  pg = wave_sum(pg);
  pdl = wave_sum(pdl);
  prr = wave_sum(prr);
  if (lane == 0) {
    s_red[t >> 6] = pg;
    s_red[16 + (t >> 6)] = pdl;
    s_red[32 + (t >> 6)] = prr;
  }
  __syncthreads();
  if (!s_flag[0]) return;
  double gam = 0.0, del = 0.0, rr = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    gam += s_red[k];
    del += s_red[16 + k];
    rr += s_red[32 + k];
  }
  const bool first = tl.idx == 0 && t == 0;
  LMState *stw = pd.st;
  if (it > 0 && sqrt(rr) <= tol * sqrt(bb)) {  // converged after it updates
    if (first) {
      stw->pcg_done = 1;
      stw->pcg_iters = it;
    }
    return;
  }
  double beta = 0.0, den = del;
  if (it > 0) {
    beta = gam / gprev;
    den = del - beta * gam / aprev;
  }
  if (!(den > 0.0)) {  // p.S p <= 0: breakdown, keep x
    if (first) {
      stw->pcg_done = 1;
      stw->pcg_iters = it + 1;
    }
    return;
  }
  const double alpha = gam / den;
  if (first) {
    stw->cg_alpha[cu] = alpha;
    stw->cg_gamma[cu] = gam;
  }
  const T ta = T(alpha), tb = T(beta);
  T *r1 = (T *)pd.cg_r[cu];
  T *u1 = (T *)pd.cg_u[cu];
  T *w1 = (T *)pd.cg_w[cu];
  T *s1 = (T *)pd.cg_s[cu];
  T *p1 = (T *)(cu ? pd.p1 : pd.p0);
  // ---- columns: s_it, r_{it+1}, u_{it+1} = M^-1 r_{it+1}; own rows also p_it, x_{it+1}
  // (own-row stores wait until after the last barrier so no barrier waits on them)
  T sm = T(0), rm = T(0), um = T(0), pn = T(0);
  if (has_col) {
    cg_column<T>(m, tb, ta, cw, cs, cr, mrow, sm, rm, um);
    ul[6 * l + m] = um;
    if (own) {
      pn = u0m + tb * p0m;
      s_ro[c - row0][m] = rm;
      s_uo[c - row0][m] = um;
    }
  }
  for (int k = t + kCgColThreads; k < 6 * ncmax && t < kCgColThreads; k += kCgColThreads) {
    const int l2 = k / 6, m2 = k - 6 * (k / 6);
    const int c2 = tcol[l2];
    if (c2 < 0) break;  // lists are -1 padded: k grows, so no later column follows
    const size_t b = 6 * (size_t)c2;
    T w2[6], s2[6], r2[6];
    double mr2[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      w2[n] = w0[b + n];
      s2[n] = s0[b + n];
      r2[n] = r0[b + n];
      mr2[n] = pd.Minv[36 * (size_t)c2 + 6 * m2 + n];
    }
    T sm2, rm2, um2;
    cg_column<T>(m2, tb, ta, w2, s2, r2, mr2, sm2, rm2, um2);
    ul[6 * l2 + m2] = um2;
    if (c2 >= row0 && c2 < row1) {
      const size_t idx = b + m2;
      const T pn2 = u0[idx] + tb * p0[idx];
      p1[idx] = pn2;
      x[idx] = x[idx] + ta * pn2;
      s1[idx] = sm2;
      r1[idx] = rm2;
      u1[idx] = um2;
      s_ro[c2 - row0][m2] = rm2;
      s_uo[c2 - row0][m2] = um2;
    }
  }
  __syncthreads();
  // ---- w_{it+1} = S u_{it+1} for the tile's rows
  T acc = T(0);
  if (spl) {
#pragma unroll
    for (int k = 0; k < kCgPre; ++k)
      if (lreg[k] >= 0) {
        const T *uc = ul + 6 * lreg[k];
#pragma unroll
        for (int n = 0; n < 6; ++n) acc += sreg[k][n] * uc[n];
      }
    for (int blk = b0 + bstep * kCgPre; blk < b1; blk += bstep) {
      const T *Srow = S + 36 * (size_t)blk + 6 * i;
      const T *uc = ul + 6 * pd.S_lcol[blk];
#pragma unroll
      for (int n = 0; n < 6; ++n) acc += Srow[n] * uc[n];
    }
  }
  T wi = T(0);
  if (Lr >= 64) {
#pragma unroll
    for (int gg = 0; gg < 10; ++gg) wi += __shfl(acc, 6 * gg + i, 64);
  } else {  // half-wave rows: the five groups of this half
    const int sbase = t & 32;
#pragma unroll
    for (int gg = 0; gg < 5; ++gg) wi += __shfl(acc, sbase + 6 * gg + i, 64);
  }
  if (hs < 6 && a < row1) s_w[rw][q][hs] = wi;
  __syncthreads();
  if (own) {
    const size_t idx = 6 * (size_t)c + m;
    p1[idx] = pn;
    x[idx] = xm + ta * pn;
    s1[idx] = sm;
    r1[idx] = rm;
    u1[idx] = um;
  }
  // ---- partials of gamma_{it+1}, delta_{it+1}, ||r_{it+1}||^2: wave 0 alone when the
  // tile's 6 R elements fit in it, else waves 0 to 3 and one more barrier
  const bool one_wave = 6 * R <= 64;
  if (one_wave ? t < 64 : t < 256) {
    double g2 = 0.0, d2 = 0.0, q2 = 0.0;
    if (t < 6 * R) {
      const int rr_ = t / 6, mm = t - 6 * (t / 6);
      const int a2 = row0 + rr_;
      if (a2 < row1) {
        T w = s_w[rr_][0][mm];
        for (int qq = 1; qq < wpr; ++qq) w += s_w[rr_][qq][mm];
        w1[6 * (size_t)a2 + mm] = w;
        const double ui = (double)s_uo[rr_][mm], ri = (double)s_ro[rr_][mm];
        g2 = ri * ui;
        d2 = (double)w * ui;
        q2 = ri * ri;
      }
    }
    g2 = wave_sum(g2);
    d2 = wave_sum(d2);
    q2 = wave_sum(q2);
    if (one_wave) {
      if (t == 0) {
        double *pn = pd.part_cg[cu];
        pn[tl.idx] = g2;
        pn[nt + tl.idx] = d2;
        pn[2 * nt + tl.idx] = q2;
      }
      return;
    }
    if ((t & 63) == 0) {
      s_fin[3 * (t >> 6)] = g2;
      s_fin[3 * (t >> 6) + 1] = d2;
      s_fin[3 * (t >> 6) + 2] = q2;
    }
  }
  if (one_wave) return;
  __syncthreads();
  if (t == 0) {
    double *pn = pd.part_cg[cu];
    pn[tl.idx] = s_fin[0] + s_fin[3] + s_fin[6] + s_fin[9];
    pn[nt + tl.idx] = s_fin[1] + s_fin[4] + s_fin[7] + s_fin[10];
    pn[2 * nt + tl.idx] = s_fin[2] + s_fin[5] + s_fin[8] + s_fin[11];
  }
}

template <class T, int RC>
__global__ __launch_bounds__(1024) void k_cg_step(const ProbDev *__restrict__ probs,
                                                  const Tile *__restrict__ tiles, int it) {
  const Tile tl = tiles[blockIdx.x];
  cg_step_body<T, RC>(probs[tl.prob], tl.idx, it);
}

// The same step for a batch of one problem, its descriptor passed by value: the
// launch saves the two dependent loads (tile table, descriptor) that precede
// every other load of the step.
template <class T, int RC>
__global__ __launch_bounds__(1024) void k_cg_step1(const ProbDev pd, int it) {
  cg_step_body<T, RC>(pd, blockIdx.x, it);
}

// Loads and stores of the values tiles of the resident PCG hand each other within one
// launch (partial sums; w, s and r of a tile's own rows): agent-coherent accesses,
// served at the device's coherence point rather than from an XCD's L2, since the L2s
// of the eight XCDs are not coherent with each other.
template <class V>
__device__ inline V ld_shared(const V *p) {
  return __hip_atomic_load(const_cast<V *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class V>
__device__ inline void st_shared(V *p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier of the resident PCG.  Each wave waits until its stores have been
// acknowledged (the shared values above are written agent-coherent, so acknowledged
// means visible to every XCD); thread 0 then sets the tile's flag, and wave 0 polls
// every tile's flag (one agent-coherent load per lane and 64 tiles) until all have
// reached `stamp`.  Readers take the shared values with agent-coherent loads issued
// after the poll, so neither an L2 write-back nor an invalidate is needed: the form
// with a release/acquire pair per workgroup measured 9.3 us per iteration with one
// counter and 8.3 us with per-tile flags, this form 7.2 us, and a launch per iteration
// 8.0 us (2M-observation drive).
// The wait is bounded: after `polls` polls (LMState::bar_polls) the workgroup reports
// failure, so a launch whose workgroups cannot all be resident at once ends instead of
// waiting forever.
__device__ inline bool grid_barrier(uint32_t *flag, int n_tiles, int tile, uint32_t stamp, int polls,
                                    int *s_ok) {
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 64) {
    if (t == 0) st_shared(flag + tile, stamp);
    bool all = false;
    for (int n = 0; n < polls; ++n) {
      // a lane's flags (up to four: 256 tiles) are loaded together, so that one poll
      // costs one round trip; a loop over them waited for each load before the next
      // (lanes past the last tile load its flag again: every load is unconditional)
      bool mine = true;
      uint32_t v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = ld_shared(flag + min(t + 64 * q, n_tiles - 1));
#pragma unroll
      for (int q = 0; q < 4; ++q) mine = mine & (v[q] >= stamp);
      for (int k = t + 256; k < n_tiles; k += 64) mine = mine & (ld_shared(flag + k) >= stamp);
      all = __all(mine) != 0;
      if (all) break;
      __builtin_amdgcn_s_sleep(1);
    }
    if (t == 0) s_ok[0] = all ? 1 : 0;
  }
  __syncthreads();
  return s_ok[0] != 0;
}

// The whole one-reduction PCG of one problem in one launch, for a grid whose tiles are
// all resident at once (checked by the host): the same iterates in the same order as
// pcg_max launches of k_cg_step1, with a grid barrier where a launch boundary was.
// What a launch re-read every iteration stays on chip for the whole solve: the tile's
// S blocks in registers (those a lane group holds; longer rows read the rest each
// iteration), the M^-1 rows of its columns in LDS, and u, p and x of its own rows in
// registers.  Per iteration a tile reads only the partial sums and w, s and r of its
// columns, and stores w, s and r of its own rows (x once at the end).  pd.cg_flag
// holds the barrier's per-tile flags, cleared by k_cg_start.

// Dynamic LDS of k_cg_run: u of the tile's columns, then their M^-1 rows (FP64).
__host__ __device__ constexpr size_t cg_run_mrow_offset(int max_tcols, size_t tbytes) {
  return (6 * (size_t)max_tcols * tbytes + 7) / 8;  // in doubles
}
size_t cg_run_lds_bytes(int max_tcols, size_t tbytes) {
  return 8 * cg_run_mrow_offset(max_tcols, tbytes) + 36 * sizeof(double) * (size_t)max_tcols;
}

template <class T, int RC>
__global__ __launch_bounds__(1024) void k_cg_run(const ProbDev pd, int n_iter) {
  extern __shared__ double s_dyn[];
  T *ul = (T *)s_dyn;  // [tile columns][6]: u_{it+1} of every column this tile reads
  // [tile columns][6][6]: M^-1 rows (in LDS: the S blocks fill the registers)
  double *ml = s_dyn + cg_run_mrow_offset(pd.max_tcols, sizeof(T));
  __shared__ double s_red[48];
  __shared__ T s_w[kPcgRowsMax][4][6];
  __shared__ T s_ro[kPcgRowsMax][6], s_uo[kPcgRowsMax][6];
  __shared__ int s_flag[2];
  const int tile = blockIdx.x;
  LMState *st = pd.st;
  const int t = threadIdx.x;
  const int nt = pd.n_pcg_tiles;
  const int R = RC ? RC : pd.pcg_rows;
  const int Lr = kCgThreads / R;
  const int wpr = Lr >= 64 ? Lr / 64 : 1;
  const int row0 = tile * R, row1 = min(pd.Cf, row0 + R);
  const int ncmax = pd.max_tcols;  // at most kCgColThreads / 6: one sweep holds every column
  const int32_t *tcol = pd.tcol + (size_t)tile * ncmax;
  const T *S = (const T *)pd.S;
  T *x = (T *)pd.x;
  if (t == 0) s_flag[0] = (lm_active(st) && !st->pcg_done) ? 1 : 0;
  __syncthreads();
  if (!s_flag[0]) return;
  n_iter = min(n_iter, st->pcg_max);
  const double tol = st->pcg_tol, bb = st->pcg_bb;
  const int polls = st->bar_polls;
  // ---- per-solve constants and the own-row state
  const int l = t / 6, m = t - 6 * (t / 6);
  const int c = (t < kCgColThreads && l < ncmax) ? tcol[l] : -1;
  const bool has_col = c >= 0;
  const bool own = has_col && c >= row0 && c < row1;
  T um = T(0), pm = T(0), xm = T(0);  // u_it, p_{it-1} (p_{-1} = 0), x_it of an own element
  if (has_col) {  // each thread reads back only the row it wrote
#pragma unroll
    for (int n = 0; n < 6; ++n) ml[6 * t + n] = pd.Minv[36 * (size_t)c + 6 * m + n];
  }
  if (own) {
    um = ((const T *)pd.cg_u[0])[6 * (size_t)c + m];
    xm = x[6 * (size_t)c + m];
  }
  const int lrs = R == kPcgRows ? 8 : (R == kPcgRowsSparse ? 6 : 5);  // log2(Lr)
  const int lane = t & 63, rw = t >> lrs;
  const int h = t & (Lr - 1);
  const int q = Lr >= 64 ? (h >> 6) : 0;
  const int hs = Lr >= 64 ? (h & 63) : h;
  const int gps = Lr >= 64 ? 10 : 5;
  const int g = hs / 6, i = hs - 6 * (hs / 6);
  const int a = row0 + rw;
  const int bstep = gps * wpr;
  const bool spl = g < gps && a < row1;
  int b0 = 0, b1 = 0;
  if (spl) {
    b0 = pd.S_rowptr[a] + gps * q + g;
    b1 = pd.S_rowptr[a + 1];
  }
  constexpr int kCgPre = sizeof(T) == 4 ? 3 : 1;  // S blocks per lane group held for the solve
  T sreg[kCgPre][6];
  int lreg[kCgPre];
#pragma unroll
  for (int k = 0; k < kCgPre; ++k) {
    const int blk = b0 + bstep * k;
    lreg[k] = -1;
    if (blk < b1) {
      lreg[k] = pd.S_lcol[blk];
#pragma unroll
      for (int n = 0; n < 6; ++n) sreg[k][n] = S[36 * (size_t)blk + 6 * i + n];
    } else {
#pragma unroll
      for (int n = 0; n < 6; ++n) sreg[k][n] = T(0);
    }
  }
  const bool first = tile == 0 && t == 0;
  double gprev = 1.0, aprev = 1.0;  // gamma_{it-1}, alpha_{it-1}
  bool ok = true;
  for (int it = 0; it < n_iter; ++it) {
    const int pr = it & 1, cu = pr ^ 1;
    // ---- partials of iteration it and the vectors of this tile's columns
    double pg = 0.0, pdl = 0.0, prr = 0.0;
    {
      const double *part = pd.part_cg[pr];
      for (int k = t; k < nt; k += kCgThreads) {
        pg += ld_shared(part + k);
        pdl += ld_shared(part + nt + k);
        prr += ld_shared(part + 2 * nt + k);
      }
    }
    T cw[6], cs[6], cr[6];
    if (has_col) {
      const T *w0 = (const T *)pd.cg_w[pr];
      const T *s0 = (const T *)pd.cg_s[pr];
      const T *r0 = (const T *)pd.cg_r[pr];
      const size_t b = 6 * (size_t)c;
#pragma unroll
      for (int n = 0; n < 6; ++n) {
        cw[n] = ld_shared(w0 + b + n);
        cs[n] = ld_shared(s0 + b + n);
        cr[n] = ld_shared(r0 + b + n);
      }
    }
    pg = wave_sum(pg);
    pdl = wave_sum(pdl);
    prr = wave_sum(prr);
    if (lane == 0) {
      s_red[t >> 6] = pg;
      s_red[16 + (t >> 6)] = pdl;
      s_red[32 + (t >> 6)] = prr;
    }
    __syncthreads();
    double gam = 0.0, del = 0.0, rr = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      gam += s_red[k];
      del += s_red[16 + k];
      rr += s_red[32 + k];
    }
    // every tile takes the same decisions from the same sums
    if (it > 0 && sqrt(rr) <= tol * sqrt(bb)) {
      if (first) {
        st->pcg_done = 1;
        st->pcg_iters = it;
      }
      break;
    }
    double beta = 0.0, den = del;
    if (it > 0) {
      beta = gam / gprev;
      den = del - beta * gam / aprev;
    }
    if (!(den > 0.0)) {
      if (first) {
        st->pcg_done = 1;
        st->pcg_iters = it + 1;
      }
      break;
    }
    const double alpha = gam / den;
    if (first) {
      st->cg_alpha[cu] = alpha;
      st->cg_gamma[cu] = gam;
    }
    gprev = gam;
    aprev = alpha;
    const T ta = T(alpha), tb = T(beta);
    // ---- columns: s_it, r_{it+1}, u_{it+1}; own rows p_it and x_{it+1}
    T sm = T(0), rm = T(0), un = T(0), pn = T(0);
    if (has_col) {
      double mrow[6];
#pragma unroll
      for (int n = 0; n < 6; ++n) mrow[n] = ml[6 * t + n];
      cg_column<T>(m, tb, ta, cw, cs, cr, mrow, sm, rm, un);
      ul[6 * l + m] = un;
      if (own) {
        pn = um + tb * pm;
        s_ro[c - row0][m] = rm;
        s_uo[c - row0][m] = un;
      }
    }
    __syncthreads();
    // ---- w_{it+1} = S u_{it+1} for the tile's rows
    T acc = T(0);
    if (spl) {
#pragma unroll
      for (int k = 0; k < kCgPre; ++k)
        if (lreg[k] >= 0) {
          const T *uc = ul + 6 * lreg[k];
#pragma unroll
          for (int n = 0; n < 6; ++n) acc += sreg[k][n] * uc[n];
        }
      for (int blk = b0 + bstep * kCgPre; blk < b1; blk += bstep) {
        const T *Srow = S + 36 * (size_t)blk + 6 * i;
        const T *uc = ul + 6 * pd.S_lcol[blk];
#pragma unroll
        for (int n = 0; n < 6; ++n) acc += Srow[n] * uc[n];
      }
    }
    T wi = T(0);
    if (Lr >= 64) {
#pragma unroll
      for (int gg = 0; gg < 10; ++gg) wi += __shfl(acc, 6 * gg + i, 64);
    } else {
      const int sbase = t & 32;
#pragma unroll
      for (int gg = 0; gg < 5; ++gg) wi += __shfl(acc, sbase + 6 * gg + i, 64);
    }
    if (hs < 6 && a < row1) s_w[rw][q][hs] = wi;
    __syncthreads();
    if (own) {
      const size_t idx = 6 * (size_t)c + m;
      st_shared((T *)pd.cg_s[cu] + idx, sm);
      st_shared((T *)pd.cg_r[cu] + idx, rm);
      pm = pn;
      xm = xm + ta * pn;
      um = un;
    }
    // ---- w_{it+1} of the tile's rows and its partials of gamma_{it+1}, delta_{it+1},
    // ||r_{it+1}||^2 (as the per-launch step: wave 0 alone when 6 R <= 64)
    const bool one_wave = 6 * R <= 64;
    if (one_wave ? t < 64 : t < 256) {
      double g2 = 0.0, d2 = 0.0, q2 = 0.0;
      if (t < 6 * R) {
        const int rr_ = t / 6, mm = t - 6 * (t / 6);
        const int a2 = row0 + rr_;
        if (a2 < row1) {
          T w = s_w[rr_][0][mm];
          for (int qq = 1; qq < wpr; ++qq) w += s_w[rr_][qq][mm];
          st_shared((T *)pd.cg_w[cu] + 6 * (size_t)a2 + mm, w);
          const double ui = (double)s_uo[rr_][mm], ri = (double)s_ro[rr_][mm];
          g2 = ri * ui;
          d2 = (double)w * ui;
          q2 = ri * ri;
        }
      }
      g2 = wave_sum(g2);
      d2 = wave_sum(d2);
      q2 = wave_sum(q2);
      if (one_wave) {
        if (t == 0) {
          double *pn2 = pd.part_cg[cu];
          st_shared(pn2 + tile, g2);
          st_shared(pn2 + nt + tile, d2);
          st_shared(pn2 + 2 * nt + tile, q2);
        }
      } else if ((t & 63) == 0) {
        s_red[3 * (t >> 6)] = g2;
        s_red[3 * (t >> 6) + 1] = d2;
        s_red[3 * (t >> 6) + 2] = q2;
      }
    }
    if (!one_wave) {
      __syncthreads();
      if (t == 0) {
        double *pn2 = pd.part_cg[cu];
        st_shared(pn2 + tile, s_red[0] + s_red[3] + s_red[6] + s_red[9]);
        st_shared(pn2 + nt + tile, s_red[1] + s_red[4] + s_red[7] + s_red[10]);
        st_shared(pn2 + 2 * nt + tile, s_red[2] + s_red[5] + s_red[8] + s_red[11]);
      }
    }
    if (!grid_barrier(pd.cg_flag, nt, tile, (uint32_t)(it + 1), polls, s_flag + 1)) {
      ok = false;
      break;
    }
  }
  if (own) x[6 * (size_t)c + m] = xm;
  if (!ok && t == 0) {
    st->pcg_fault = 1;
    st->pcg_done = 1;
  }
}

// The step kernels of one compute type for a launch whose problems all tile their rows
// by R (0: mixed, read per problem).
template <class T>
struct CgStep {
  static const void *multi(int R) {
    switch (R) {
      case kPcgRows: return (const void *)k_cg_step<T, kPcgRows>;
      case kPcgRowsSparse: return (const void *)k_cg_step<T, kPcgRowsSparse>;
      case kPcgRowsMax: return (const void *)k_cg_step<T, kPcgRowsMax>;
      default: return (const void *)k_cg_step<T, 0>;
    }
  }
  static const void *single(int R) {
    switch (R) {
      case kPcgRows: return (const void *)k_cg_step1<T, kPcgRows>;
      case kPcgRowsSparse: return (const void *)k_cg_step1<T, kPcgRowsSparse>;
      case kPcgRowsMax: return (const void *)k_cg_step1<T, kPcgRowsMax>;
      default: return (const void *)k_cg_step1<T, 0>;
    }
  }
  static const void *resident(int R) {
    switch (R) {
      case kPcgRows: return (const void *)k_cg_run<T, kPcgRows>;
      case kPcgRowsSparse: return (const void *)k_cg_run<T, kPcgRowsSparse>;
      case kPcgRowsMax: return (const void *)k_cg_run<T, kPcgRowsMax>;
      default: return (const void *)k_cg_run<T, 0>;
    }
  }
};

// ------------------------------------------------------------------ camera update
template <class T>
__global__ __launch_bounds__(256) void k_cam_update(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  __shared__ double s_red[4];
  const int cur = st->cur;
  const double lam = st->lambda;
  const int c = tl.idx * kCamTile + threadIdx.x;
  double dl = 0.0;
  if (c < pd.C) {
    const double *src = pd.pose[cur] + 12 * c;
    double *dst = pd.pose[1 - cur] + 12 * c;
    const int a = pd.free_idx[c];
    if (a < 0) {
      for (int i = 0; i < 12; ++i) dst[i] = src[i];
    } else {
      const T *x = (const T *)pd.x + 6 * a;
      const T *gc = (const T *)pd.gc + 6 * a;
      const T *Dc = (const T *)pd.Dc + 6 * a;
      double xi[6];
      for (int i = 0; i < 6; ++i) {
        xi[i] = (double)x[i];
        dl += lam * (double)Dc[i] * xi[i] * xi[i] - (double)gc[i] * xi[i];
      }
      double dR[9], dt[3];
      se3_exp(xi, dR, dt);
      for (int r = 0; r < 3; ++r) {
        for (int cc = 0; cc < 3; ++cc)
          dst[3 * r + cc] = dR[3 * r] * src[cc] + dR[3 * r + 1] * src[3 + cc] + dR[3 * r + 2] * src[6 + cc];
        dst[9 + r] = dR[3 * r] * src[9] + dR[3 * r + 1] * src[10] + dR[3 * r + 2] * src[11] + dt[r];
      }
    }
  }
  const double tot = block_sum256(dl, s_red);
  if (threadIdx.x == 0) pd.part_dl_cam[tl.idx] = tot;
}

// ------------------------------------------------------------------ point back-substitution + trial cost
template <class T, class S>
__global__ __launch_bounds__(kObsChunk) void k_point_trial(const ProbDev *__restrict__ probs,
                                                     const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int cur = st->cur;
  const double lam = st->lambda;
  const T delta = T(st->huber_delta);
  const int j0 = tl.idx * pd.pt_tile;
  const int j1 = min(pd.P, j0 + pd.pt_tile);
  const int k0 = pd.pt_start[j0], k1 = pd.pt_start[j1];
  __shared__ T s_acc[kPtTile][3];
  __shared__ T s_c[kObsChunk][3];
  __shared__ int s_loc[kObsChunk];
  __shared__ double s_X[kPtTile][3];
  __shared__ double s_red[kObsChunk / 64];
  for (int i = threadIdx.x; i < kPtTile * 3; i += kObsChunk) (&s_acc[0][0])[i] = T(0);
  const auto lin = as_global((const LinRec<T, S> *)pd.lin);
  const auto x = as_global((const T *)pd.x);
  const auto obs_pt = as_global(pd.obs_pt), obs_cam = as_global(pd.obs_cam), obs_rpos = as_global(pd.obs_rpos);
  const auto obs_act = as_global((const uint8_t *)pd.obs_act);
  const auto free_idx = as_global(pd.free_idx);
  __syncthreads();
  // phase 1: sum_k W_k^T dc_{cam(k)} = sum_k J_p^T (J_c dc) per point
  for (int base = k0; base < k1; base += kObsChunk) {
    const int k = base + threadIdx.x;
    T c[3] = {T(0), T(0), T(0)};
    int jl = -1;
    if (k < k1) {
      jl = obs_pt[k] - j0;
      const int cpos = obs_rpos[k];
      if (cpos >= 0) {
        const int cam = obs_cam[k];
        const int a = free_idx[cam];
        T f[7], R[9], Jc[12], Jp[6];
        const LinRec<T, S> rec = load_rec(lin + cpos);
        decode(rec, f);
        load_rot(pd.pose[cur] + 12 * cam, R);  // the linearisation state
        jc_from(f, Jc);
        jp_from(f, R, Jp);
        const auto dc = x + 6 * a;
        T u0 = T(0), u1 = T(0);
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          const T d = dc[m];
          u0 += Jc[m] * d;
          u1 += Jc[6 + m] * d;
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) c[m] = Jp[m] * u0 + Jp[3 + m] * u1;
      }
    }
    seg_add_scan<T, 3>(c, jl, s_acc, s_c, s_loc);
  }
  // phase 2: dp_j, trial point, point part of the predicted decrease
  const auto Vinv = as_global((const T *)pd.Vinv);
  const auto gp = as_global((const T *)pd.gp);
  const auto Dp = as_global((const T *)pd.Dp);
  double dl = 0.0;
  for (int jl = threadIdx.x; jl < j1 - j0; jl += kObsChunk) {
    const int j = j0 + jl;
    const auto vi = Vinv + 6 * (size_t)j;
    const T M[9] = {vi[0], vi[1], vi[2], vi[1], vi[3], vi[4], vi[2], vi[4], vi[5]};
    T rhs[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) rhs[i] = -gp[3 * j + i] - s_acc[jl][i];
    const auto X = as_global((const double *)pd.X[cur]) + 3 * (size_t)j;
    const auto Xn = as_global(pd.X[1 - cur]) + 3 * (size_t)j;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T d = M[3 * i] * rhs[0] + M[3 * i + 1] * rhs[1] + M[3 * i + 2] * rhs[2];
      const double dd = (double)d;
      dl += lam * (double)Dp[3 * j + i] * dd * dd - (double)gp[3 * j + i] * dd;
      const double v = X[i] + dd;
      Xn[i] = v;
      s_X[jl][i] = v;
    }
  }
  __syncthreads();
  // phase 3: trial cost at (T', X')
  const auto Kall = as_global((const T *)pd.K);
  const auto uv = as_global((const T *)pd.obs_uv);
  const auto poses = as_global((const double *)pd.pose[1 - cur]);
  double cost = 0.0;
  int masked = 0;
  for (int k = k0 + threadIdx.x; k < k1; k += kObsChunk) {
    if (!obs_act[k]) continue;
    const int jl = obs_pt[k] - j0;
    const int cam = obs_cam[k];
    double xd, yd, zd;
    transform(poses + 12 * cam, s_X[jl], xd, yd, zd);
    T r0, r1;
    if (residual<T>(Kall + 4 * cam, T(xd), T(yd), T(zd), uv[2 * (size_t)k], uv[2 * (size_t)k + 1], r0, r1))
      cost += 0.5 * (double)huber_rho(r0 * r0 + r1 * r1, delta);
    else
      ++masked;
  }
  const double tc = block_sum_w<kObsChunk / 64>(cost, s_red);
  const double td = block_sum_w<kObsChunk / 64>(dl, s_red);
  const double tm = block_sum_w<kObsChunk / 64>((double)masked, s_red);
  if (threadIdx.x == 0) {
    pd.part_trial_cost[tl.idx] = tc;
    pd.part_dl_pt[tl.idx] = td;
    pd.part_trial_masked[tl.idx] = (int32_t)tm;
  }
}

// ------------------------------------------------------------------ LM control
// One workgroup per problem.  Madsen-Nielsen-Tingleff damping: accept iff the
// gain ratio exceeds 1e-3, the predicted decrease is positive and the step puts
// no further observation behind its camera; on accept
// lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; on reject lambda *= nu, nu *= 2.
__global__ __launch_bounds__(256) void k_lm_control(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  __shared__ double s_red[4];
  __shared__ double s_red6[6][4];
  // prior terms first, so that no tile sum below is live across their loops
  double pc = 0.0, pt = 0.0;
  const bool pri = pd.rig_mode == 1 || pd.prior_on;
  if (pd.rig_mode == 1) {  // the rig priors at the current (first call only) and trial poses
    if (!st->init_done) pc = prior_cost(pd, pd.rig_pose[st->cur], s_red);
    pt = prior_cost(pd, pd.rig_pose[1 - st->cur], s_red);
  } else if (pd.prior_on) {  // the same, summed over k_prior_cost's tiles
    const int n = pd.n_pri_tiles;
    pc = block_sum_array(pd.part_prior, n, s_red);
    pt = block_sum_array(pd.part_prior + n, n, s_red);
  }
  // the tile sums, each in the order of block_sum_array (thread-strided, then the
  // four waves in order), all loaded in one pass and reduced through one barrier
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // lin cost, trial cost, dl_pt, masked, trial masked, dl_cam
  {
    // a thread's loads of kU strides are all issued before its sums, which run in
    // index order (loads past the end read the last tile and add nothing)
    constexpr int kU = 8;
    const int n = pd.n_pt_tiles;
    for (int i0 = threadIdx.x; i0 < n; i0 += 256 * kU) {
      double l0[kU], l1[kU], l2[kU];
      int32_t m0[kU], m1[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = min(i0 + 256 * u, n - 1);
        l0[u] = pd.part_lin_cost[i];
        l1[u] = pd.part_trial_cost[i];
        l2[u] = pd.part_dl_pt[i];
        m0[u] = pd.part_masked[i];
        m1[u] = pd.part_trial_masked[i];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (i0 + 256 * u < n) {
          v[0] += l0[u];
          v[1] += l1[u];
          v[2] += l2[u];
          v[3] += (double)m0[u];
          v[4] += (double)m1[u];
        }
    }
  }
  for (int i = threadIdx.x; i < pd.n_cam_tiles; i += 256) v[5] += pd.part_dl_cam[i];
  {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double x = wave_sum(v[q]);
      if (lane == 0) s_red6[q][w] = x;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double sum6[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) sum6[q] = s_red6[q][0] + s_red6[q][1] + s_red6[q][2] + s_red6[q][3];
  double c0 = sum6[0], tc = sum6[1];
  if (pri) {
    if (!st->init_done) c0 += pc;
    tc += pt;
  }
  const double dlp = sum6[2], m0 = sum6[3], mt = sum6[4], dlc = sum6[5];
  const int n = st->iter;
  if (!st->init_done) {
    st->cost = c0;
    st->cost0 = c0;
    st->n_masked = (int32_t)m0;
    st->init_done = 1;
    pd.iter_cost[0] = c0;
  }
  const double C = st->cost;
  const double dL = 0.5 * (dlc + dlp);
  const double rho = (dL != 0.0) ? (C - tc) / dL : -INFINITY;
  st->trial_cost = tc;
  st->dL = dL;
  st->rho = rho;
  double lam = st->lambda;
  pd.iter_pcg[n] = st->pcg_done ? st->pcg_iters : st->pcg_max;
  // a step that puts more observations behind their cameras is rejected
  const bool more_masked = (int32_t)mt > st->n_masked;
  const bool fault = st->pcg_fault != 0;  // the step is not a PCG result: reject it and stop
  if (!fault && isfinite(tc) && dL > 0.0 && rho > kAcceptRho && !more_masked) {
    st->cost = tc;
    st->n_masked = (int32_t)mt;
    st->cur = 1 - st->cur;
    const double t = 2.0 * rho - 1.0;
    lam *= fmax(1.0 / 3.0, 1.0 - t * t * t);
    st->nu = 2.0;
    st->relin = 1;
    st->accepted += 1;
  } else {
    lam *= st->nu;
    st->nu *= 2.0;
    st->relin = 0;
  }
  lam = fmin(fmax(lam, kLambdaMin), kLambdaMax);
  st->lambda = lam;
  pd.iter_cost[n + 1] = st->cost;
  st->pcg_done = 0;
  st->pcg_iters = 0;
  st->iter = n + 1;
  if (fault) st->halted = 1;  // the remaining iterations do nothing
  if (st->iter >= st->max_iters || fault) {
    if (fault) st->status = 3;
    else if (!isfinite(st->cost)) st->status = 2;
    else if (lam >= kLambdaMax) st->status = 1;
    else st->status = 0;
  }
}

// ------------------------------------------------------------------ evaluation
// sum ||r||^2 and the masked count at the accepted state, per point tile.
template <class T>
__global__ __launch_bounds__(256) void k_eval(const ProbDev *__restrict__ probs,
                                              const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  const int cur = st->cur;
  const int j0 = tl.idx * pd.pt_tile;
  const int j1 = min(pd.P, j0 + pd.pt_tile);
  const int k0 = pd.pt_start[j0], k1 = pd.pt_start[j1];
  const T *Kall = (const T *)pd.K;
  const T *uv = (const T *)pd.obs_uv;
  __shared__ double s_red[4];
  double sq = 0.0;
  int masked = 0;
  for (int k = k0 + threadIdx.x; k < k1; k += 256) {
    if (!pd.obs_act[k]) continue;
    const int j = pd.obs_pt[k];
    const int cam = pd.obs_cam[k];
    double xd, yd, zd;
    transform(pd.pose[cur] + 12 * cam, pd.X[cur] + 3 * (size_t)j, xd, yd, zd);
    T r0, r1;
    if (residual<T>(Kall + 4 * cam, T(xd), T(yd), T(zd), uv[2 * (size_t)k], uv[2 * (size_t)k + 1], r0, r1))
      sq += (double)(r0 * r0 + r1 * r1);
    else
      ++masked;
  }
  const double tsq = block_sum256(sq, s_red);
  const double tm = block_sum256((double)masked, s_red);
  if (threadIdx.x == 0) {
    pd.part_sq[tl.idx] = tsq;
    pd.part_masked[tl.idx] = (int32_t)tm;
  }
}

// ------------------------------------------------------------------ culling and re-triangulation
// The step between BA rounds of the iterative triangulation framework (Sec. 4.3).
// At the accepted state an active observation stays iff its point is in front of
// the camera and ||r||^2 <= tau2 (residual in FP64 from the stored pixels).  A point
// that lost an observation is re-triangulated from the active ones that remain by
// the multi-view midpoint method; it leaves the problem (all its observations
// inactive) when fewer than two remain or the triangulation fails.  One thread per
// point; per-tile counts of active observations and of points with at least one
// go to part_cull.

// Triangulation of one point from observations given by get(k, P, x, y): false if
// observation k is not used, else the world -> camera pose P (12 values) and the
// normalized image coordinates (x, y) = K^-1 (u, v).  Both methods run in FP64 and fail
// when an observation that is used would see the point at depth <= kZMin.
template <class Get>
__device__ inline bool tri_depths_ok(int n, Get get, const double X[3]) {
  for (int k = 0; k < n; ++k) {
    const double *P;
    double x, y;
    if (!get(k, P, x, y)) continue;
    if (!(P[6] * X[0] + P[7] * X[1] + P[8] * X[2] + P[11] > kZMin)) return false;
  }
  return true;
}

// Midpoint: the X minimising the summed squared distances to the observation rays, the
// solution of (sum_k (I - d_k d_k^T)) X = sum_k (I - d_k d_k^T) c_k with centre
// c_k = -R^T t and unit ray d_k along R^T (x, y, 1), by the adjugate.  Fails when the 3x3
// determinant is <= 1e-12.
template <class Get>
__device__ bool tri_midpoint(int n, Get get, double out[3]) {
  double A[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // xx, xy, xz, yy, yz, zz
  double b[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < n; ++k) {
    const double *P;
    double a0, a1;
    if (!get(k, P, a0, a1)) continue;
    double d[3], c[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      d[m] = P[m] * a0 + P[3 + m] * a1 + P[6 + m];
      c[m] = -(P[m] * P[9] + P[3 + m] * P[10] + P[6 + m] * P[11]);
    }
    const double inv = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
    for (int m = 0; m < 3; ++m) d[m] *= inv;
    A[0] += 1.0 - d[0] * d[0];
    A[1] -= d[0] * d[1];
    A[2] -= d[0] * d[2];
    A[3] += 1.0 - d[1] * d[1];
    A[4] -= d[1] * d[2];
    A[5] += 1.0 - d[2] * d[2];
    const double dc = d[0] * c[0] + d[1] * c[1] + d[2] * c[2];
#pragma unroll
    for (int m = 0; m < 3; ++m) b[m] += c[m] - d[m] * dc;
  }
  const double c00 = A[3] * A[5] - A[4] * A[4];
  const double c01 = A[2] * A[4] - A[1] * A[5];
  const double c02 = A[1] * A[4] - A[2] * A[3];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(det > 1e-12)) return false;
  const double c11 = A[0] * A[5] - A[2] * A[2];
  const double c12 = A[1] * A[2] - A[0] * A[4];
  const double c22 = A[0] * A[3] - A[1] * A[1];
  const double id = 1.0 / det;
  out[0] = (c00 * b[0] + c01 * b[1] + c02 * b[2]) * id;
  out[1] = (c01 * b[0] + c11 * b[1] + c12 * b[2]) * id;
  out[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * id;
  return tri_depths_ok(n, get, out);
}

// DLT (the classical homogeneous form): each observation contributes the rows
// x P_3 - P_1 and y P_3 - P_2 of A; X~ is the unit eigenvector of A^T A (4x4, FP64) for
// its smallest eigenvalue, found by cyclic Jacobi rotations (8 sweeps), and
// X = X~[:3] / X~[3].  Fails when |X~[3]| <= 1e-12.
template <class Get>
__device__ bool tri_dlt(int n, Get get, double out[3]) {
  double M[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) M[a][b] = 0.0;
  for (int k = 0; k < n; ++k) {
    const double *P;
    double x, y;
    if (!get(k, P, x, y)) continue;
    // P rows: (R_r0, R_r1, R_r2, t_r)
    double r1[4], r2[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r1[c] = x * P[6 + c] - P[c];
      r2[c] = y * P[6 + c] - P[3 + c];
    }
    r1[3] = x * P[11] - P[9];
    r2[3] = y * P[11] - P[10];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) M[a][b] += r1[a] * r1[b] + r2[a] * r2[b];
  }
  double V[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) V[a][b] = a == b ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 8; ++sweep)
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        const double apq = M[p][q];
        if (apq == 0.0) continue;
        const double tau = (M[q][q] - M[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < 4; ++k) {  // columns p, q of M
          const double mkp = M[k][p], mkq = M[k][q];
          M[k][p] = c * mkp - s * mkq;
          M[k][q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < 4; ++k) {  // rows p, q of M
          const double mpk = M[p][k], mqk = M[q][k];
          M[p][k] = c * mpk - s * mqk;
          M[q][k] = s * mpk + c * mqk;
        }
        for (int k = 0; k < 4; ++k) {  // columns p, q of V
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  int mi = 0;
  for (int a = 1; a < 4; ++a)
    if (M[a][a] < M[mi][mi]) mi = a;
  const double w = V[3][mi];
  if (!(fabs(w) > 1e-12)) return false;
  out[0] = V[0][mi] / w;
  out[1] = V[1][mi] / w;
  out[2] = V[2][mi] / w;
  return tri_depths_ok(n, get, out);
}

template <class T>
__global__ __launch_bounds__(256) void k_cull(const ProbDev *__restrict__ probs,
                                              const Tile *__restrict__ tiles, double tau2, int method) {
  static_assert(kPtTile == 256, "one thread per point of the largest tile");
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const int cur = pd.st->cur;
  const int j = tl.idx * pd.pt_tile + (int)threadIdx.x;
  __shared__ double s_red[4];
  int n_act = 0;
  if ((int)threadIdx.x < pd.pt_tile && j < pd.P) {
    const int k0 = pd.pt_start[j], k1 = pd.pt_start[j + 1];
    const T *Kall = (const T *)pd.K;
    const T *uv = (const T *)pd.obs_uv;
    const double *poses = pd.pose[cur];
    double *X = pd.X[cur] + 3 * (size_t)j;
    const double Xj[3] = {X[0], X[1], X[2]};
    bool lost = false;
    for (int k = k0; k < k1; ++k) {
      if (!pd.obs_act[k]) continue;
      const int cam = pd.obs_cam[k];
      const T *K = Kall + 4 * cam;
      double x, y, z;
      transform(poses + 12 * cam, Xj, x, y, z);
      bool keep = z > kZMin;
      if (keep) {
        const double r0 = (double)K[0] * x / z + (double)K[2] - (double)uv[2 * (size_t)k];
        const double r1 = (double)K[1] * y / z + (double)K[3] - (double)uv[2 * (size_t)k + 1];
        keep = r0 * r0 + r1 * r1 <= tau2;
      }
      if (keep) {
        ++n_act;
      } else {
        pd.obs_act[k] = 0;
        lost = true;
      }
    }
    if (lost) {
      double Xn[3];
      auto get = [&](int kk, const double *&P, double &x, double &y) {
        const int k = k0 + kk;
        if (!pd.obs_act[k]) return false;
        const int cam = pd.obs_cam[k];
        const T *K = Kall + 4 * cam;
        P = poses + 12 * cam;
        x = ((double)uv[2 * (size_t)k] - (double)K[2]) / (double)K[0];
        y = ((double)uv[2 * (size_t)k + 1] - (double)K[3]) / (double)K[1];
        return true;
      };
      const bool ok = n_act >= 2 && (method == 1 ? tri_dlt(k1 - k0, get, Xn) : tri_midpoint(k1 - k0, get, Xn));
      if (ok) {
        X[0] = Xn[0];
        X[1] = Xn[1];
        X[2] = Xn[2];
      } else {
        for (int k = k0; k < k1; ++k) pd.obs_act[k] = 0;
        n_act = 0;
      }
    }
  }
  const double ta = block_sum256((double)n_act, s_red);
  const double tp = block_sum256(n_act > 0 ? 1.0 : 0.0, s_red);
  if (threadIdx.x == 0) {
    pd.part_cull[2 * tl.idx] = (int32_t)ta;
    pd.part_cull[2 * tl.idx + 1] = (int32_t)tp;
  }
}

// ------------------------------------------------------------------ vehicle-rig BA
// Sec. 4.4: the pose of rig camera c at frame f is E_c T_v(f).  The composed-camera
// view forms the undamped reduced system S_cam, b_cam over the cameras (f, c) with the
// BA kernels; the rig increments map to camera increments as
//   xi_(f,c) = Ad(E_c) xi_v(f) + xi_e(c)      (E Exp(xi) E^-1 = Exp(Ad(E) xi)),
// i.e. xi_cam = B xi_rig, so the rig system is S_rig = B^T S_cam B, b_rig = B^T b_cam,
// g_rig = B^T g_cam and the rig Hessian's diagonal blocks are B^T U_cam B.  The rig
// view adds its priors (extrinsic absolute prior, rigidity pairs), damps with the
// Marquardt diagonal of the rig Hessian and runs the PCG; the update moves vehicles and
// extrinsics, recomposes the cameras and hands xi_cam = B xi_rig to the points.
constexpr int kMaxRigCams = 16;

// Ad(E) = [[R, [t]x R], [0, R]] for E = (R, t) held as 12 values, acting on (rho, phi).
__device__ inline void rig_adjoint(const double *E, double A[36]) {
  double H[9];
  hat3(E + 9, H);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[6 * i + j] = E[3 * i + j];
      A[6 * i + 3 + j] = H[3 * i] * E[j] + H[3 * i + 1] * E[3 + j] + H[3 * i + 2] * E[6 + j];
      A[6 * (i + 3) + j] = 0.0;
      A[6 * (i + 3) + 3 + j] = E[3 * i + j];
    }
}

// Rig blocks of S_rig = B^T S_cam B in two passes.  k_rig_seg: one wave per segment of
// at most kRigSeg contributions of one rig block; lane (i, j) < 36 holds element
// (i, j); each contribution L^T S_ab R of a camera block, with L, R = Ad(E_c) for a
// vehicle side and the identity for an extrinsic side, is formed as S R then L^T (S R)
// through lane shuffles, every S block of the segment loaded before the arithmetic,
// and the segment's sum goes to rpart in FP64.  k_rig_blocks: one wave per rig block
// sums its segments in order and writes the off-diagonal blocks to S and the undamped
// diagonal ones to rdiag.
template <class T>
__global__ __launch_bounds__(256) void k_rig_seg(const ProbDev *__restrict__ probs,
                                                 const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  __shared__ double s_ad[kMaxRigCams][36];
  const int nr = pd.n_rigcam;
  if ((int)threadIdx.x < nr) {
    double A[36];
    rig_adjoint(pd.pose[st->cur] + 12 * (size_t)(pd.n_frames + threadIdx.x), A);
    for (int e = 0; e < 36; ++e) s_ad[threadIdx.x][e] = A[e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int sg = 4 * tl.idx + w;
  if (sg >= pd.n_rig_seg) return;  // no barrier follows
  const int i = min(lane / 6, 5), j = lane - 6 * (lane / 6);
  const T *Sc = (const T *)pd.cam_S;
  const int c0 = pd.rs_c0[sg], n = pd.rs_c0[sg + 1] - c0;
  double acc = 0.0;
  for (int g0 = 0; g0 < n; g0 += 8) {  // eight contributions loaded before their arithmetic
    double sv[8];
    int lr[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const bool live = g0 + h < n;
      lr[h] = live ? pd.rb_lr[c0 + g0 + h] : 0;
      sv[h] = (live && lane < 36) ? (double)Sc[36 * (size_t)pd.rb_pos[c0 + g0 + h] + lane] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      if (g0 + h < n) {  // uniform across the wave
        const int lc = (lr[h] & 0xffff) - 1, rc = (lr[h] >> 16) - 1;
        double t1 = sv[h];
        if (rc >= 0) {  // (S R)_ij = sum_l S_il R_lj
          t1 = 0.0;
#pragma unroll
          for (int l = 0; l < 6; ++l) t1 += __shfl(sv[h], 6 * i + l, 64) * s_ad[rc][6 * l + j];
        }
        double o = t1;
        if (lc >= 0) {  // (L^T T1)_ij = sum_k L_ki T1_kj
          o = 0.0;
#pragma unroll
          for (int k = 0; k < 6; ++k) o += s_ad[lc][6 * k + i] * __shfl(t1, 6 * k + j, 64);
        }
        acc += o;
      }
    }
  }
  if (lane < 36) pd.rpart[36 * (size_t)sg + lane] = acc;
}

template <class T>
__global__ __launch_bounds__(256) void k_rig_blocks(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = 4 * tl.idx + w;
  if (b >= pd.nnzb || lane >= 36) return;
  const int s0 = pd.rs_blk[b], s1 = pd.rs_blk[b + 1];
  double acc = 0.0;
  for (int sg = s0; sg < s1; sg += 8) {  // eight partials in flight, summed in order
    double v[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) v[h] = sg + h < s1 ? pd.rpart[36 * (size_t)(sg + h) + lane] : 0.0;
#pragma unroll
    for (int h = 0; h < 8; ++h) acc += v[h];
  }
  const int dr = pd.rb_diag[b];
  if (dr >= 0)
    pd.rdiag[36 * (size_t)dr + lane] = acc;
  else
    ((T *)pd.S)[36 * (size_t)b + lane] = T(acc);
}

// Row sums of one free rig unknown, one wave: over its composed cameras (a vehicle: the
// rig cameras of its frame, through Ad(E_c); an extrinsic: its camera at every frame)
// the Hessian block B^T U B (21), g (6) and b (6) in FP64, lane-strided then summed by a
// fixed butterfly; then the 54-value row [U | U - S_diag | g | b + g] that
// finish_camera_row turns into the damped diagonal block, the right-hand side b and the
// block-Jacobi inverse.
template <class T>
__global__ __launch_bounds__(64) void k_rig_rows(const ProbDev *__restrict__ probs,
                                                 const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int x = tl.idx;
  const int nr = pd.n_rigcam;
  const bool vehicle = pd.free_cam[x] < pd.n_frames;
  const int lane = threadIdx.x;
  const T *gc = (const T *)pd.cam_gc;
  const T *bc = (const T *)pd.cam_brhs;
  double acc[33];
  for (int e = 0; e < 33; ++e) acc[e] = 0.0;
  for (int k = pd.rr_start[x] + lane; k < pd.rr_start[x + 1]; k += 64) {
    const int cam = pd.rr_cam[k];
    const double *Uu = pd.cam_U + 21 * (size_t)cam;
    double U[36], g[6], bb[6];
    int u = 0;
    for (int r = 0; r < 6; ++r)
      for (int c = r; c < 6; ++c, ++u) U[6 * r + c] = U[6 * c + r] = Uu[u];
    for (int r = 0; r < 6; ++r) {
      g[r] = (double)gc[6 * (size_t)cam + r];
      bb[r] = (double)bc[6 * (size_t)cam + r];
    }
    if (vehicle) {
      double A[36], UA[36];
      rig_adjoint(pd.pose[st->cur] + 12 * (size_t)(pd.n_frames + cam % nr), A);
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          double v = 0.0;
          for (int m = 0; m < 6; ++m) v += U[6 * r + m] * A[6 * m + c];
          UA[6 * r + c] = v;
        }
      u = 0;
      for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c, ++u) {
          double v = 0.0;
          for (int m = 0; m < 6; ++m) v += A[6 * m + r] * UA[6 * m + c];
          acc[u] += v;
        }
      for (int r = 0; r < 6; ++r) {
        double vg = 0.0, vb = 0.0;
        for (int m = 0; m < 6; ++m) {
          vg += A[6 * m + r] * g[m];
          vb += A[6 * m + r] * bb[m];
        }
        acc[21 + r] += vg;
        acc[27 + r] += vb;
      }
    } else {
      for (int e = 0; e < 21; ++e) acc[e] += Uu[e];
      for (int r = 0; r < 6; ++r) {
        acc[21 + r] += g[r];
        acc[27 + r] += bb[r];
      }
    }
  }
  for (int e = 0; e < 33; ++e) acc[e] = wave_sum(acc[e]);
  if (lane == 0) {
    double *o = pd.row_tot + 54 * (size_t)x;
    const double *Sd = pd.rdiag + 36 * (size_t)x;
    int u = 0;
    for (int r = 0; r < 6; ++r)
      for (int c = r; c < 6; ++c, ++u) {
        o[u] = acc[u];
        o[21 + u] = acc[u] - Sd[6 * r + c];
      }
    for (int r = 0; r < 6; ++r) {
      o[42 + r] = acc[21 + r];
      o[48 + r] = acc[27 + r] + acc[21 + r];
    }
  }
}

// Rig update and recomposition, over the composed-camera view's camera tiles: thread g
// moves rig node g (T <- Exp(xi) T for a free one, a copy for a fixed one) into the
// trial buffer with its part of the predicted decrease, and composes trial camera g
// (frame g / nr, rig camera g % nr) from the same trial vehicle and extrinsic, with its
// increment xi_cam = Ad(E_c) xi_v + xi_e for the point back-substitution.
template <class T>
__global__ __launch_bounds__(256) void k_rig_update(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  LMState *st = pd.st;
  if (!lm_active(st)) return;
  __shared__ double s_red[4];
  const int cur = st->cur;
  const double lam = st->lambda;
  const int F = pd.n_frames, nr = pd.n_rigcam;
  const T *xr = (const T *)pd.rig_x;
  const int g = tl.idx * kCamTile + threadIdx.x;
  auto trial = [&](int node, double out[12]) {
    const double *src = pd.rig_pose[cur] + 12 * (size_t)node;
    const int a = pd.rig_free_idx[node];
    if (a < 0) {
      for (int i = 0; i < 12; ++i) out[i] = src[i];
      return;
    }
    double xi[6], dR[9], dt[3];
    for (int i = 0; i < 6; ++i) xi[i] = (double)xr[6 * (size_t)a + i];
    se3_exp(xi, dR, dt);
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c)
        out[3 * r + c] = dR[3 * r] * src[c] + dR[3 * r + 1] * src[3 + c] + dR[3 * r + 2] * src[6 + c];
      out[9 + r] = dR[3 * r] * src[9] + dR[3 * r + 1] * src[10] + dR[3 * r + 2] * src[11] + dt[r];
    }
  };
  double dl = 0.0;
  if (g < F + nr) {
    double Tn[12];
    trial(g, Tn);
    double *dst = pd.rig_pose[1 - cur] + 12 * (size_t)g;
    for (int i = 0; i < 12; ++i) dst[i] = Tn[i];
    const int a = pd.rig_free_idx[g];
    if (a >= 0) {
      const T *gr = (const T *)pd.rig_gc + 6 * (size_t)a;
      const T *Dr = (const T *)pd.rig_Dc + 6 * (size_t)a;
      for (int i = 0; i < 6; ++i) {
        const double xi = (double)xr[6 * (size_t)a + i];
        dl += lam * (double)Dr[i] * xi * xi - (double)gr[i] * xi;
      }
    }
  }
  if (g < pd.C) {
    const int f = g / nr, c = g - nr * (g / nr);
    double Tv[12], Te[12];
    trial(f, Tv);
    trial(F + c, Te);
    double *dst = pd.pose[1 - cur] + 12 * (size_t)g;
    for (int r = 0; r < 3; ++r) {
      for (int cc = 0; cc < 3; ++cc)
        dst[3 * r + cc] = Te[3 * r] * Tv[cc] + Te[3 * r + 1] * Tv[3 + cc] + Te[3 * r + 2] * Tv[6 + cc];
      dst[9 + r] = Te[3 * r] * Tv[9] + Te[3 * r + 1] * Tv[10] + Te[3 * r + 2] * Tv[11] + Te[9 + r];
    }
    double xc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int av = pd.rig_free_idx[f], ae = pd.rig_free_idx[F + c];
    if (av >= 0) {
      double A[36];
      rig_adjoint(pd.rig_pose[cur] + 12 * (size_t)(F + c), A);
      for (int r = 0; r < 6; ++r)
        for (int m = 0; m < 6; ++m) xc[r] += A[6 * r + m] * (double)xr[6 * (size_t)av + m];
    }
    if (ae >= 0)
      for (int r = 0; r < 6; ++r) xc[r] += (double)xr[6 * (size_t)ae + r];
    T *xo = (T *)pd.x + 6 * (size_t)g;
    for (int r = 0; r < 6; ++r) xo[r] = T(xc[r]);
  }
  const double tot = block_sum256(dl, s_red);
  if (threadIdx.x == 0) pd.part_dl_cam[tl.idx] = tot;
}

// ------------------------------------------------------------------ pose-only Gauss-Newton
// One workgroup per request; the whole iteration count runs in the kernel.
// FP32 projection and Jacobians, FP32 per-thread sums of H (21) and g (6)
// combined in FP64, FP64 6x6 Cholesky solve and FP64 pose update.
__global__ __launch_bounds__(kPoseThreads) void k_pose_gn(PoseDev *__restrict__ reqs,
                                                          const double *__restrict__ Xall,
                                                          const float *__restrict__ uvall) {
  PoseDev &rq = reqs[blockIdx.x];
  const int iters = rq.iters;
  const float delta = (float)rq.delta;
  __shared__ double s_pose[12];
  __shared__ double s_sum[4][28];
  __shared__ int s_bad;
  if (threadIdx.x < 12) s_pose[threadIdx.x] = rq.pose[threadIdx.x];
  if (threadIdx.x == 0) s_bad = 0;
  const float K[4] = {(float)rq.K[0], (float)rq.K[1], (float)rq.K[2], (float)rq.K[3]};
  const double *X = Xall + 3 * rq.off;
  const float *uv = uvall + 2 * rq.off;
  const int n = rq.n;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  for (int it = 0; it <= iters; ++it) {
    float acc[28];
#pragma unroll
    for (int i = 0; i < 28; ++i) acc[i] = 0.0f;
    double cost = 0.0;
    double pose[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) pose[i] = s_pose[i];
    for (int c = threadIdx.x; c < n; c += kPoseThreads) {
      double xd, yd, zd;
      transform(pose, X + 3 * (size_t)c, xd, yd, zd);
      const float x = (float)xd, y = (float)yd, z = (float)zd;
      float r0, r1;
      if (!residual<float>(K, x, y, z, uv[2 * c], uv[2 * c + 1], r0, r1)) continue;
      const float s = r0 * r0 + r1 * r1;
      cost += 0.5 * (double)huber_rho(s, delta);
      if (it == iters) continue;
      const float wgt = huber_w(s, delta);
      float Jc[12], Jp[6];
      jacobians<float>(K, pose, x, y, z, Jc, Jp);
      int u = 0;
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int cc = r; cc < 6; ++cc, ++u) acc[u] += wgt * (Jc[r] * Jc[cc] + Jc[6 + r] * Jc[6 + cc]);
#pragma unroll
      for (int r = 0; r < 6; ++r) acc[21 + r] += wgt * (Jc[r] * r0 + Jc[6 + r] * r1);
    }
    acc[27] = 0.0f;
    double dacc[28];
#pragma unroll
    for (int i = 0; i < 27; ++i) dacc[i] = wave_sum((double)acc[i]);
    dacc[27] = wave_sum(cost);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < 28; ++i) s_sum[w][i] = dacc[i];
    __syncthreads();
    if (threadIdx.x == 0) {
      // every loop below has constant bounds and is unrolled, so that the 6x6 solve
      // stays in registers (with its arrays indexed at run time it ran from scratch
      // memory)
      double tot[28];
#pragma unroll
      for (int i = 0; i < 28; ++i) tot[i] = s_sum[0][i] + s_sum[1][i] + s_sum[2][i] + s_sum[3][i];
      if (it == iters) {
        rq.cost = tot[27];
      } else {
        double H[36];
        {
          int u = 0;
#pragma unroll
          for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int cc = r; cc < 6; ++cc, ++u) {
              H[6 * r + cc] = tot[u];
              H[6 * cc + r] = tot[u];
            }
        }
        // Cholesky solve H d = -g; a non-positive pivot marks the system singular (the
        // columns after it are formed with a unit pivot and not used)
        double L[36];
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 36; ++i) L[i] = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          double s = H[7 * j];
#pragma unroll
          for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
          ok = ok && s > 0.0;
          L[7 * j] = ok ? sqrt(s) : 1.0;
#pragma unroll
          for (int i = j + 1; i < 6; ++i) {
            double t = H[6 * i + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = t / L[7 * j];
          }
        }
        if (!ok) {
          s_bad = 1;
        } else {
          double yv[6], d[6];
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            double s = -tot[21 + i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= L[6 * i + k] * yv[k];
            yv[i] = s / L[7 * i];
          }
#pragma unroll
          for (int i = 5; i >= 0; --i) {
            double s = yv[i];
#pragma unroll
            for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * d[k];
            d[i] = s / L[7 * i];
          }
          double dR[9], dt[3], np[12];
          se3_exp(d, dR, dt);
#pragma unroll
          for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              np[3 * r + cc] = dR[3 * r] * s_pose[cc] + dR[3 * r + 1] * s_pose[3 + cc] + dR[3 * r + 2] * s_pose[6 + cc];
            np[9 + r] = dR[3 * r] * s_pose[9] + dR[3 * r + 1] * s_pose[10] + dR[3 * r + 2] * s_pose[11] + dt[r];
          }
#pragma unroll
          for (int i = 0; i < 12; ++i) s_pose[i] = np[i];
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 12) rq.pose[threadIdx.x] = s_pose[threadIdx.x];
  if (threadIdx.x == 0) rq.status = s_bad;
}

// ------------------------------------------------------------------ dense co-visibility form
// For scenes where every camera sees most points, S is dense and the pair lists of the
// sparse forms would outgrow memory (a point seen by L free cameras has L (L - 1) / 2
// pairs).  This form never lists pairs.  With V*_j = L_j L_j^T (Cholesky of the damped
// point block) each observation's 6x3 block Z_aj = W_aj L_j^-T, W_aj = J_c^T J_p, gives
//   sum_j W_aj V*_j^-1 W_bj^T = sum_j Z_aj Z_bj^T   and   sum_j W_aj V*_j^-1 g_p,j = sum_j Z_aj h_j
// with h_j = L_j^-1 g_p,j: S - U* is a Gram matrix over the points' three directions,
// a dense contraction that runs on the matrix cores.  Workgroup (tile pair (ta, tb),
// point range) builds Z for its 16 + 16 cameras and 32 points at a time in LDS and
// accumulates the 96 x 96 product Z_ta Z_tb^T with MFMA; the ranges' partial products
// are summed in a fixed order by k_dense_reduce.

// Per point: V* = V + lambda D_p, its inverse (back-substitution), and L^-T (upper:
// 00 01 02 11 12 22) and h = L^-1 g_p of its Cholesky factor, in FP64.
template <class T>
__global__ __launch_bounds__(256) void k_dense_prep(const ProbDev *__restrict__ probs,
                                                    const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int j = tl.idx * pd.pt_tile + (int)threadIdx.x;
  if ((int)threadIdx.x >= pd.pt_tile || j >= pd.P) return;
  const double lam = st->lambda;
  const T *V = (const T *)pd.V;
  const T *Dp = (const T *)pd.Dp;
  const T *gp = (const T *)pd.gp;
  double u[6], o[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) u[i] = (double)V[6 * (size_t)j + i];
  u[0] += lam * (double)Dp[3 * (size_t)j + 0];
  u[3] += lam * (double)Dp[3 * (size_t)j + 1];
  u[5] += lam * (double)Dp[3 * (size_t)j + 2];
  inv_sym3(u, o);
  T *Vinv = (T *)pd.Vinv + 6 * (size_t)j;
#pragma unroll
  for (int i = 0; i < 6; ++i) Vinv[i] = T(o[i]);
  const double l00 = sqrt(fmax(u[0], 1e-300));
  const double l10 = u[1] / l00, l20 = u[2] / l00;
  const double l11 = sqrt(fmax(u[3] - l10 * l10, 1e-300));
  const double l21 = (u[4] - l20 * l10) / l11;
  const double l22 = sqrt(fmax(u[5] - l20 * l20 - l21 * l21, 1e-300));
  // M = L^-1 (lower triangular)
  const double m00 = 1.0 / l00, m11 = 1.0 / l11, m22 = 1.0 / l22;
  const double m10 = -l10 * m00 * m11, m21 = -l21 * m11 * m22;
  const double m20 = -(l20 * m00 + l21 * m10) * m22;
  const double g0 = (double)gp[3 * (size_t)j], g1 = (double)gp[3 * (size_t)j + 1], g2 = (double)gp[3 * (size_t)j + 2];
  T *pf = (T *)pd.dn_pfac + 9 * (size_t)j;
  pf[0] = T(m00);
  pf[1] = T(m10);
  pf[2] = T(m20);
  pf[3] = T(m11);
  pf[4] = T(m21);
  pf[5] = T(m22);
  pf[6] = T(m00 * g0);
  pf[7] = T(m10 * g0 + m11 * g1);
  pf[8] = T(m20 * g0 + m21 * g1 + m22 * g2);
}

// Z (6x3) of one observation: W = J_c^T J_p times the point's L^-T (lt, upper).
template <class T>
__device__ inline void dense_z(const T Jc[12], const T Jp[6], const T lt[6], T Z[18]) {
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const T w0 = Jc[m] * Jp[0] + Jc[6 + m] * Jp[3];
    const T w1 = Jc[m] * Jp[1] + Jc[6 + m] * Jp[4];
    const T w2 = Jc[m] * Jp[2] + Jc[6 + m] * Jp[5];
    Z[3 * m] = w0 * lt[0];
    Z[3 * m + 1] = w0 * lt[1] + w1 * lt[3];
    Z[3 * m + 2] = w0 * lt[2] + w1 * lt[4] + w2 * lt[5];
  }
}

// Camera sums of the dense form, one workgroup per free camera over its observations
// (camera-major list): U (21), g_c (6) and sum_j Z_aj h_j (6), per thread in the
// compute type, then in FP64 in a fixed order into the camera's row sums.
constexpr int kDnCamThreads = 1024;
template <class T, class S>
__global__ __launch_bounds__(kDnCamThreads) void k_dense_cams(const ProbDev *__restrict__ probs,
                                                              const Tile *__restrict__ tiles) {
  constexpr bool k16 = sizeof(S) == 2;
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int a = tl.idx;
  const int cam = pd.free_cam[a];
  const double *pose = pd.pose[st->cur] + 12 * cam;
  T R[9];
  load_rot(pose, R);
  const T *K = (const T *)pd.K + 4 * cam;
  const T delta = T(st->huber_delta);
  const LinRec<T, S> *lin = (const LinRec<T, S> *)pd.lin;
  const T *pf = (const T *)pd.dn_pfac;
  T acc[33];
#pragma unroll
  for (int i = 0; i < 33; ++i) acc[i] = T(0);
  for (int o = pd.cam_obs_start[a] + (int)threadIdx.x; o < pd.cam_obs_start[a + 1]; o += kDnCamThreads) {
    const int2 cr = pd.dn_crec[o];  // record position, point
    const int j = cr.y;
    const LinRec<T, S> rec = lin[cr.x];
    T f[7], Jc[12], Jp[6], lt[6], hv[3], Z[18];
    decode(rec, f);
    jc_from(f, Jc);
    jp_from(f, R, Jp);
#pragma unroll
    for (int i = 0; i < 6; ++i) lt[i] = pf[9 * (size_t)j + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) hv[i] = pf[9 * (size_t)j + 6 + i];
    acc_jtj_upper(acc, Jc);
    if (k16) {
      // 16-bit storage: the gradient from FP32 Jacobians at the linearisation state
      const int k = pd.cam_obs[o];
      double xd, yd, zd;
      transform(pose, pd.X[st->cur] + 3 * (size_t)j, xd, yd, zd);
      const T xv = T(xd), yv = T(yd), zv = T(zd);
      const T *uv = (const T *)pd.obs_uv + 2 * (size_t)k;
      T r0, r1;
      if (pd.obs_act[k] && residual<T>(K, xv, yv, zv, uv[0], uv[1], r0, r1)) {
        const T w = huber_w(r0 * r0 + r1 * r1, delta);
        T Jg[12], Jpg[6];
        jacobians<T>(K, pose, xv, yv, zv, Jg, Jpg);
#pragma unroll
        for (int r = 0; r < 6; ++r) acc[21 + r] += w * (Jg[r] * r0 + Jg[6 + r] * r1);
      }
    } else {
      const T e0 = rec.e[0], e1 = rec.e[1];
#pragma unroll
      for (int r = 0; r < 6; ++r) acc[21 + r] += Jc[r] * e0 + Jc[6 + r] * e1;
    }
    dense_z(Jc, Jp, lt, Z);
#pragma unroll
    for (int m = 0; m < 6; ++m) acc[27 + m] += Z[3 * m] * hv[0] + Z[3 * m + 1] * hv[1] + Z[3 * m + 2] * hv[2];
  }
  constexpr int NW = kDnCamThreads / 64;
  __shared__ double s_t[NW][33];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 33; ++i) {
    const double v = wave_sum((double)acc[i]);
    if (lane == 0) s_t[wv][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < 33) {
    const int i = threadIdx.x;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += s_t[w][i];
    // row sums: U (0..20), sum Y W^T (21..41, from k_dense_reduce), g_c (42..47), Y g_p (48..53)
    pd.row_tot[54 * (size_t)a + (i < 21 ? i : 21 + i)] = v;
  }
}

// Operand type E of the products, k-values per MFMA instruction KI and points per chunk
// PC of each (compute, storage) pair: FP64 and FP32 products in their own type
// (16x16x4), FP16 / BF16 storage with 16-bit operands (16x16x32, FP32 accumulation).
typedef float dn_f4 __attribute__((ext_vector_type(4)));
typedef double dn_d4 __attribute__((ext_vector_type(4)));
typedef _Float16 dn_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 dn_b8 __attribute__((ext_vector_type(8)));
template <class T, class S>
struct DnMma;
template <>
struct DnMma<double, double> {
  using E = double;
  using V = dn_d4;
  static constexpr int KI = 4, PC = 16;
  static constexpr bool row_major_d = false;  // D[i][j]: lane j + 16 (i % 4), register i / 4
  __device__ static V mma(const E *a, const E *b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(*a, *b, c, 0, 0, 0); }
};
template <>
struct DnMma<float, float> {
  using E = float;
  using V = dn_f4;
  static constexpr int KI = 4, PC = 16;
  static constexpr bool row_major_d = true;   // D[i][j]: lane j + 16 (i / 4), register i % 4
  __device__ static V mma(const E *a, const E *b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0); }
};
template <>
struct DnMma<float, _Float16> {
  using E = _Float16;
  using V = dn_f4;
  static constexpr int KI = 32, PC = 32;
  static constexpr bool row_major_d = true;
  __device__ static V mma(const E *a, const E *b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(*(const dn_h8 *)a, *(const dn_h8 *)b, c, 0, 0, 0);
  }
};
template <>
struct DnMma<float, bf16s> {
  using E = __bf16;
  using V = dn_f4;
  static constexpr int KI = 32, PC = 32;
  static constexpr bool row_major_d = true;
  __device__ static V mma(const E *a, const E *b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const dn_b8 *)a, *(const dn_b8 *)b, c, 0, 0, 0);
  }
};
// LDS layout of a Z tile in k_dense_schur: k-value kk of row r at
// (kk / KI) * kDnRows * RS + r * RS + kk % KI, where a camera's six rows are spread
// (row m of camera slot a at kDnCams * m + a), so that the 16 cameras a wave stores at
// once fall in distinct banks, and a row holds KI values plus, for 16-bit operands, 8 of
// padding, so that the 16-byte operand reads of 16 consecutive rows do not share banks.
template <class T, class S>
constexpr int dn_row_stride() {
  return DnMma<T, S>::KI + (sizeof(typename DnMma<T, S>::E) == 2 ? 8 : 0);
}
// Dynamic LDS of k_dense_schur: two Z tiles of 3 PC k-values by kDnRows rows.
template <class T, class S>
constexpr size_t dn_lds_bytes() {
  return 2 * (size_t)(3 * DnMma<T, S>::PC / DnMma<T, S>::KI) * kDnRows * dn_row_stride<T, S>() *
         sizeof(typename DnMma<T, S>::E);
}

// Tile pair (ta <= tb) of a pair index, row-major over the upper triangle of nt tiles.
__device__ inline void dn_pair(int pair, int nt, int &ta, int &tb) {
  int a = 0, rem = pair;
  while (rem >= nt - a) {
    rem -= nt - a;
    ++a;
  }
  ta = a;
  tb = a + rem;
}

// One (tile pair, point range): Z tiles in LDS laid out [k / KI][row][k % KI] so that
// the 64 lanes of an operand load read one contiguous run; four waves, each a 48 x 48
// quarter of the 96 x 96 product (3 x 3 MFMA tiles of 16 x 16).  Thread (point jl,
// sub) owns camera slots sub, sub + SUB, ... of its point in each tile and writes their
// Z blocks, or zeros where the camera does not see the point (the point's camera mask
// gives presence and the record's place in the point's range).  The records of the next
// chunk are loaded into registers before the current chunk's products, so their latency
// hides behind the matrix cores.
template <class T, class S>
__global__ __launch_bounds__(256) void k_dense_schur(const ProbDev *__restrict__ probs,
                                                     const Tile *__restrict__ tiles) {
  using M = DnMma<T, S>;
  using E = typename M::E;
  using V = typename M::V;
  constexpr int KI = M::KI, PC = M::PC, K = 3 * PC, NKS = K / KI, SUB = 256 / PC, KL = KI / 4;
  constexpr int NSLOT = kDnCams / SUB;  // camera slots of one point and tile per thread
  constexpr int RS = dn_row_stride<T, S>(), BS = kDnRows * RS;  // row and k-block strides
  extern __shared__ __align__(16) double s_dyn[];
  E *za = (E *)s_dyn;        // [NKS][kDnRows][RS]
  E *zb = za + NKS * BS;     // the same for tile tb (unused when ta == tb)
  __shared__ T s_R[2][kDnCams][9];
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int pair = tl.idx / pd.dn_split, split = tl.idx - pair * pd.dn_split;
  int ta, tb;
  dn_pair(pair, pd.dn_tiles, ta, tb);
  const bool diag = ta == tb;
  const int nsides = diag ? 1 : 2;
  const int nt = pd.dn_tiles, nt1 = pd.dn_tiles + 1;
  const int t = threadIdx.x;
  if (t < 2 * kDnCams) {
    const int side = t / kDnCams, la = t - kDnCams * side;
    const int a = (side ? tb : ta) * kDnCams + la;
    T R[9];
    if (a < pd.Cf) {
      load_rot(pd.pose[st->cur] + 12 * pd.free_cam[a], R);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = T(0);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) s_R[side][la][i] = R[i];
  }
  const int j0 = (int)((int64_t)pd.P * split / pd.dn_split);
  const int j1 = (int)((int64_t)pd.P * (split + 1) / pd.dn_split);
  const LinRec<T, S> *lin = (const LinRec<T, S> *)pd.lin;
  const T *pf = (const T *)pd.dn_pfac;
  const int lane = t & 63, wv = t >> 6;
  const int rb0 = 3 * (wv >> 1), cb0 = 3 * (wv & 1);
  const int li = lane & 15, lq = lane >> 4;
  const int jl = t / SUB, sub = t - SUB * (t / SUB);
  // the next chunk's records of this thread's camera slots (stored Jacobian values)
  S nf[2][NSLOT][7];
  bool npr[2][NSLOT];
  T nlt[6];
  auto fetch = [&](int jc) {
    const int j = jc + jl;
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int q = 0; q < NSLOT; ++q) npr[side][q] = false;
    if (j >= j1) return;
#pragma unroll
    for (int i = 0; i < 6; ++i) nlt[i] = pf[9 * (size_t)j + i];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side >= nsides) break;
      const int tt = side ? tb : ta;
      const int r0 = pd.dn_ts[(size_t)j * nt1 + tt];
      const uint32_t mk = pd.dn_mask[(size_t)j * nt + tt];
#pragma unroll
      for (int q = 0; q < NSLOT; ++q) {
        const int la = sub + SUB * q;
        if ((mk >> la) & 1u) {
          const int r = r0 + __popc(mk & ((1u << la) - 1u));
#pragma unroll
          for (int i = 0; i < 7; ++i) nf[side][q][i] = lin[r].f[i];
          npr[side][q] = true;
        }
      }
    }
  };
  V acc[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[r][c][e] = 0;
  fetch(j0);
  for (int jc = j0; jc < j1; jc += PC) {
    __syncthreads();  // the previous chunk's products are done (and s_R is visible)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side >= nsides) break;
      E *z = side ? zb : za;
#pragma unroll
      for (int q = 0; q < NSLOT; ++q) {
        const int la = sub + SUB * q;
        T Z[18];
        if (npr[side][q]) {
          T f[7], Jc[12], Jp[6];
#pragma unroll
          for (int i = 0; i < 7; ++i) f[i] = Codec<S>::dec(nf[side][q][i]);
          jc_from(f, Jc);
          jp_from(f, &s_R[side][la][0], Jp);
          dense_z(Jc, Jp, nlt, Z);
        } else {
#pragma unroll
          for (int i = 0; i < 18; ++i) Z[i] = T(0);
        }
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int kk = 3 * jl + c, row = kDnCams * m + la;
            z[(kk / KI) * BS + row * RS + (kk % KI)] = E(Z[3 * m + c]);
          }
      }
    }
    __syncthreads();
    if (jc + PC < j1) fetch(jc + PC);  // in flight during the products below
    const E *zbb = diag ? za : zb;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const E *ab = za + ks * BS + li * RS + lq * KL;
      const E *bb = zbb + ks * BS + li * RS + lq * KL;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          acc[r][c] = M::mma(ab + 16 * (rb0 + r) * RS, bb + 16 * (cb0 + c) * RS, acc[r][c]);
    }
  }
  T *out = (T *)pd.dn_part + (size_t)tl.idx * kDnRows * kDnRows;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // LDS rows back to camera-major rows (6 per camera)
        const int prow = 16 * (rb0 + r) + (M::row_major_d ? 4 * lq + e : lq + 4 * e);
        const int pcol = 16 * (cb0 + c) + li;
        const int row = 6 * (prow % kDnCams) + prow / kDnCams;
        const int col = 6 * (pcol % kDnCams) + pcol / kDnCams;
        out[row * kDnRows + col] = T(acc[r][c][e]);
      }
}

// One camera row (6 rows) of one tile pair: the ranges' partial products summed in FP64
// in range order; blocks (a < b) go to S as -sum and its transpose, diagonal blocks'
// upper halves to the camera's row sums (sum Y W^T), finished with the other sums by
// k_schur_finish.  Tile index = pair * kDnCams + row camera.
template <class T>
__global__ __launch_bounds__(256) void k_dense_reduce(const ProbDev *__restrict__ probs,
                                                      const Tile *__restrict__ tiles) {
  const Tile tl = tiles[blockIdx.x];
  const ProbDev &pd = probs[tl.prob];
  const LMState *st = pd.st;
  if (!lm_active(st)) return;
  const int pair = tl.idx / kDnCams, lr = tl.idx - kDnCams * pair;
  int ta, tb;
  dn_pair(pair, pd.dn_tiles, ta, tb);
  const int a = ta * kDnCams + lr;
  if (a >= pd.Cf) return;
  const int ns = pd.dn_split;
  constexpr int NE = kDnRows * kDnRows;
  const T *part = (const T *)pd.dn_part + (size_t)pair * ns * NE + 6 * lr * kDnRows;
  T *Sv = (T *)pd.S;
  for (int e = threadIdx.x; e < 6 * kDnRows; e += 256) {
    const int r = e / kDnRows, Cc = e - kDnRows * (e / kDnRows);
    const int b = tb * kDnCams + Cc / 6;
    if (b >= pd.Cf || a > b) continue;  // a > b: written as a transpose
    double sum = 0.0;
    for (int x = 0; x < ns; ++x) sum += (double)part[(size_t)x * NE + e];
    const int c = Cc % 6;
    if (a == b) {
      if (r <= c) pd.row_tot[54 * (size_t)a + 21 + 6 * r - r * (r - 1) / 2 + (c - r)] = sum;
    } else {
      const T v = T(-sum);
      Sv[36 * ((size_t)pd.S_rowptr[a] + b) + 6 * r + c] = v;
      Sv[36 * ((size_t)pd.S_rowptr[b] + a) + 6 * c + r] = v;
    }
  }
}

// ------------------------------------------------------------------ launchers
namespace {
struct Timed {
  KernelTimer *t;
  int id;
  hipStream_t s;
  Timed(KernelTimer *t_, int id_, hipStream_t s_, int launches = 1) : t(t_), id(id_), s(s_) {
    if (t) t->begin(id, s, launches);
  }
  ~Timed() {
    if (t) t->end(id, s);
  }
};
}  // namespace

// LDS available to the fused PCG form for z (bytes): the device's per-workgroup
// limit less room for the kernel's static LDS, set once by prepare_kernels().
static size_t g_fused_lds = 48 * 1024;
// Per-workgroup LDS of the device (0 when the chunk form cannot be used).
static size_t g_lds_limit = 0;
// Whether the dense form's product kernel may use its LDS on this device.
static bool g_dense_ok = false;

int prepare_kernels() {
  static bool done = false;
  if (done) return 0;
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return -1;
  size_t use = lim > 8192 ? (size_t)lim - 4096 : 0;
  if (use > 48 * 1024) {
    // dynamic LDS beyond 48 KB must be allowed per kernel
    bool ok = true;
    for (int R : {0, kPcgRows, kPcgRowsSparse, kPcgRowsMax})
      for (const void *f : {CgStep<float>::multi(R), CgStep<double>::multi(R), CgStep<float>::single(R),
                            CgStep<double>::single(R), CgStep<float>::resident(R), CgStep<double>::resident(R)})
        ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)use) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      use = 48 * 1024;
    }
  }
  g_fused_lds = use;
  g_lds_limit = lim > 0 ? (size_t)lim : 0;
  // the chunk form stages a chunk in up to chunk_lds_bytes of dynamic LDS
  const void *chunk_kernels[4] = {(const void *)k_schur_chunk<double, double>,
                                  (const void *)k_schur_chunk<float, float>,
                                  (const void *)k_schur_chunk<float, _Float16>,
                                  (const void *)k_schur_chunk<float, bf16s>};
  for (int p = 0; p < 4; ++p) {
    const size_t need = chunk_lds_bytes(p);
    if (need + 4096 > g_lds_limit ||
        hipFuncSetAttribute(chunk_kernels[p], hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) !=
            hipSuccess) {
      (void)hipGetLastError();
      g_lds_limit = 0;  // chunk form unavailable on this device
    }
  }
  // the dense form's product kernel
  const void *dense_kernels[4] = {(const void *)k_dense_schur<double, double>,
                                  (const void *)k_dense_schur<float, float>,
                                  (const void *)k_dense_schur<float, _Float16>,
                                  (const void *)k_dense_schur<float, bf16s>};
  const size_t dense_lds[4] = {dn_lds_bytes<double, double>(), dn_lds_bytes<float, float>(),
                               dn_lds_bytes<float, _Float16>(), dn_lds_bytes<float, bf16s>()};
  g_dense_ok = true;
  for (int p = 0; p < 4; ++p)
    if (dense_lds[p] + 4096 > (size_t)lim ||
        hipFuncSetAttribute(dense_kernels[p], hipFuncAttributeMaxDynamicSharedMemorySize, (int)dense_lds[p]) !=
            hipSuccess) {
      (void)hipGetLastError();
      g_dense_ok = false;
    }
  done = true;
  return 0;
}

// With no device present (an analysis for planning), the forms are chosen as for a
// gfx950 device: 160 KB of LDS per workgroup, so both the chunk and the dense form fit.
constexpr size_t kGfx950Lds = 160 * 1024;

bool dense_form_available() { return prepare_kernels() == 0 ? g_dense_ok : true; }

size_t device_lds_limit() {
  if (prepare_kernels() != 0) return kGfx950Lds;
  return g_lds_limit;
}

bool one_reduction_pcg(int precision, int max_tcols) {
  return 6 * (size_t)max_tcols * (precision == 0 ? 8 : 4) <= g_fused_lds;
}

bool resident_pcg_fits(int precision, int rows, int n_tiles, int max_tcols) {
  if (prepare_kernels() != 0 || !one_reduction_pcg(precision, max_tcols)) return false;
  if (6 * max_tcols > kCgColThreads || n_tiles < 1) return false;
  const void *f = precision == 0 ? CgStep<double>::resident(rows) : CgStep<float>::resident(rows);
  const size_t lds = cg_run_lds_bytes(max_tcols, precision == 0 ? 8 : 4);
  if (lds > g_fused_lds) return false;
  int dev = 0, n_cu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kCgThreads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (int64_t)n_tiles <= (int64_t)n_cu * per_cu;
}

template <class T, class S>
static hipError_t lm_iteration(const BatchPlan &bp, int pcg_max, int max_tcols, hipStream_t s,
                               KernelTimer *tm, int part) {
  const bool before = part == LM_ALL || part == LM_BEFORE_PCG;
  const bool pcg = part == LM_ALL || part == LM_PCG;
  const bool after = part == LM_ALL || part == LM_AFTER_PCG;
  const size_t ubytes = 6 * (size_t)max_tcols * sizeof(T);
  const bool one_reduction = ubytes <= g_fused_lds;
  if (before) {
  if (bp.n_pt) {
    Timed t(tm, K_LINEARIZE, s);
    k_linearize<T, S><<<bp.n_pt, kObsChunk, 0, s>>>(bp.probs, bp.pt);
  }
  if (bp.n_pri) {
    Timed t(tm, K_PRIOR_LIN, s);
    k_prior_lin<T><<<bp.n_pri, 256, 0, s>>>(bp.probs, bp.pri);
  }
  if (bp.n_ch) {
    Timed t(tm, K_SCHUR_CHUNK, s);
    k_schur_chunk<T, S><<<bp.n_ch, chunk_threads<T>(), chunk_lds_bytes(sizeof(T) == 8 ? 0 : 1), s>>>(bp.probs,
                                                                                                 bp.ch);
  }
  if (bp.n_red) {
    Timed t(tm, K_SCHUR_REDUCE, s);
    k_schur_reduce<T><<<bp.n_red, 256, 0, s>>>(bp.probs, bp.red);
  }
  if (bp.n_dpt) {
    Timed t(tm, K_DENSE_PREP, s);
    k_dense_prep<T><<<bp.n_dpt, 256, 0, s>>>(bp.probs, bp.dpt);
  }
  if (bp.n_dcm) {
    Timed t(tm, K_DENSE_CAMS, s);
    k_dense_cams<T, S><<<bp.n_dcm, kDnCamThreads, 0, s>>>(bp.probs, bp.dcm);
  }
  if (bp.n_dsy) {
    Timed t(tm, K_DENSE_SCHUR, s);
    k_dense_schur<T, S><<<bp.n_dsy, 256, dn_lds_bytes<T, S>(), s>>>(bp.probs, bp.dsy);
  }
  if (bp.n_dre) {
    Timed t(tm, K_DENSE_REDUCE, s);
    k_dense_reduce<T><<<bp.n_dre, 256, 0, s>>>(bp.probs, bp.dre);
  }
  if (bp.n_fin) {
    Timed t(tm, K_SCHUR_ROWS, s);
    k_schur_rows<T><<<bp.n_fin, 1024, 0, s>>>(bp.probs, bp.fin);
  }
  if (bp.n_fsh) {
    Timed t(tm, K_SCHUR_FINISH, s);
    k_schur_finish<T><<<bp.n_fsh, 64, 0, s>>>(bp.probs, bp.fsh);
  }
  if (bp.n_pp) {
    Timed t(tm, K_POINT_PREP, s);
    k_point_prep<T, S><<<bp.n_pp, 256, 0, s>>>(bp.probs, bp.pp);
  }
  if (bp.n_diag) {
    Timed t(tm, K_SCHUR_DIAG, s);
    k_schur_diag<T, S><<<bp.n_diag, 256, 0, s>>>(bp.probs, bp.diag);
  }
  if (bp.n_off) {
    Timed t(tm, K_SCHUR_OFF, s);
    k_schur_off<T, S><<<bp.n_off, 256, 0, s>>>(bp.probs, bp.off);
  }
  if (bp.n_pri) {
    Timed t(tm, K_PRIOR_APPLY, s);
    k_prior_apply<T><<<bp.n_pri, 256, 0, s>>>(bp.probs, bp.pri);
  }
  if (bp.n_pcg && one_reduction) {
    Timed t(tm, K_PCG_SPMV, s);
    if (bp.pcg_rows >= kPcgRowsSparse)
      k_cg_start<T, 16><<<bp.n_pcg, 1024, 0, s>>>(bp.probs, bp.pcg);
    else
      k_cg_start<T, 4><<<bp.n_pcg, 256, 0, s>>>(bp.probs, bp.pcg);
  }
  }
  if (pcg && bp.n_pcg && one_reduction) {
    // one event pair around the whole run: per-launch events would add their own
    // overhead to launches this short
    const bool resident = bp.n_probs == 1 && bp.single.pcg_resident;
    Timed t(tm, K_PCG_CG, s, resident ? 1 : pcg_max);
    hipError_t le = hipSuccess;
    if (resident) {
      const void *f = CgStep<T>::resident(bp.pcg_rows);
      void *args[] = {(void *)&bp.single, (void *)&pcg_max};
      const unsigned lds = (unsigned)cg_run_lds_bytes(max_tcols, sizeof(T));
      // cooperative: the runtime places every workgroup at once or fails the launch;
      // otherwise the occupancy count made at set-up stands, and in both cases the grid
      // barrier's bounded wait turns starvation into a reported status
      le = bp.single.pcg_resident == 2
               ? hipLaunchCooperativeKernel(f, dim3(bp.n_pcg), dim3(kCgThreads), args, lds, s)
               : hipLaunchKernel(f, dim3(bp.n_pcg), dim3(kCgThreads), args, lds, s);
    } else if (bp.n_probs == 1) {
      const void *f = CgStep<T>::single(bp.pcg_rows);
      for (int it = 0; it < pcg_max && le == hipSuccess; ++it) {
        void *args[] = {(void *)&bp.single, (void *)&it};
        le = hipLaunchKernel(f, dim3(bp.n_pcg), dim3(kCgThreads), args, ubytes, s);
      }
    } else {
      const void *f = CgStep<T>::multi(bp.pcg_rows);
      for (int it = 0; it < pcg_max && le == hipSuccess; ++it) {
        void *args[] = {(void *)&bp.probs, (void *)&bp.pcg, (void *)&it};
        le = hipLaunchKernel(f, dim3(bp.n_pcg), dim3(kCgThreads), args, ubytes, s);
      }
    }
    if (le != hipSuccess) return le;
  } else if (pcg) {
    for (int it = 0; it < pcg_max && bp.n_pcg; ++it) {
      {
        Timed t(tm, K_PCG_SPMV, s);
        k_pcg_spmv<T><<<bp.n_pcg, 256, 0, s>>>(bp.probs, bp.pcg, it);
      }
      {
        Timed t(tm, K_PCG_UPDATE, s);
        k_pcg_update<T><<<bp.n_pcg, 256, 0, s>>>(bp.probs, bp.pcg, it);
      }
    }
  }
  if (after) {
  if (bp.n_cam) {
    Timed t(tm, K_CAM_UPDATE, s);
    k_cam_update<T><<<bp.n_cam, 256, 0, s>>>(bp.probs, bp.cam);
  }
  if (bp.n_pt) {
    Timed t(tm, K_POINT_TRIAL, s);
    k_point_trial<T, S><<<bp.n_pt, kObsChunk, 0, s>>>(bp.probs, bp.pt);
  }
  if (bp.n_pri) {
    Timed t(tm, K_PRIOR_COST, s);
    k_prior_cost<<<bp.n_pri, 256, 0, s>>>(bp.probs, bp.pri);
  }
  if (bp.n_ctl) {
    Timed t(tm, K_LM_CONTROL, s);
    k_lm_control<<<bp.n_ctl, 256, 0, s>>>(bp.probs, bp.ctl);
  }
  }
  return hipGetLastError();
}

// One LM iteration of a vehicle-rig problem (see the vehicle-rig kernels).
template <class T, class S>
static hipError_t rig_iteration(const BatchPlan &cp, const BatchPlan &rp, int pcg_max, int max_tcols,
                                hipStream_t s, KernelTimer *tm) {
  const size_t ubytes = 6 * (size_t)max_tcols * sizeof(T);
  const bool one_reduction = ubytes <= g_fused_lds;
  // composed cameras: linearisation and the undamped reduced system
  if (cp.n_pt) {
    Timed t(tm, K_LINEARIZE, s);
    k_linearize<T, S><<<cp.n_pt, kObsChunk, 0, s>>>(cp.probs, cp.pt);
  }
  if (cp.n_ch) {
    Timed t(tm, K_SCHUR_CHUNK, s);
    k_schur_chunk<T, S><<<cp.n_ch, chunk_threads<T>(), chunk_lds_bytes(sizeof(T) == 8 ? 0 : 1), s>>>(cp.probs,
                                                                                                 cp.ch);
  }
  if (cp.n_red) {
    Timed t(tm, K_SCHUR_REDUCE, s);
    k_schur_reduce<T><<<cp.n_red, 256, 0, s>>>(cp.probs, cp.red);
  }
  if (cp.n_fin) {
    Timed t(tm, K_SCHUR_ROWS, s);
    k_schur_rows<T><<<cp.n_fin, 1024, 0, s>>>(cp.probs, cp.fin);
  }
  if (cp.n_fsh) {
    Timed t(tm, K_SCHUR_FINISH, s);
    k_schur_finish<T><<<cp.n_fsh, 64, 0, s>>>(cp.probs, cp.fsh);
  }
  if (cp.n_pp) {
    Timed t(tm, K_POINT_PREP, s);
    k_point_prep<T, S><<<cp.n_pp, 256, 0, s>>>(cp.probs, cp.pp);
  }
  if (cp.n_diag) {
    Timed t(tm, K_SCHUR_DIAG, s);
    k_schur_diag<T, S><<<cp.n_diag, 256, 0, s>>>(cp.probs, cp.diag);
  }
  if (cp.n_off) {
    Timed t(tm, K_SCHUR_OFF, s);
    k_schur_off<T, S><<<cp.n_off, 256, 0, s>>>(cp.probs, cp.off);
  }
  // rig unknowns: priors, projection, damping, preconditioner, PCG
  if (rp.n_pri) {
    Timed t(tm, K_PRIOR_LIN, s);
    k_prior_lin<T><<<rp.n_pri, 256, 0, s>>>(rp.probs, rp.pri);
  }
  if (rp.n_ch) {
    Timed t(tm, K_RIG_BLOCKS, s);
    k_rig_seg<T><<<rp.n_ch, 256, 0, s>>>(rp.probs, rp.ch);
  }
  if (rp.n_red) {
    Timed t(tm, K_RIG_BLOCKS, s);
    k_rig_blocks<T><<<rp.n_red, 256, 0, s>>>(rp.probs, rp.red);
  }
  if (rp.n_fin) {
    Timed t(tm, K_RIG_ROWS, s);
    k_rig_rows<T><<<rp.n_fin, 64, 0, s>>>(rp.probs, rp.fin);
  }
  if (rp.n_fsh) {
    Timed t(tm, K_SCHUR_FINISH, s);
    k_schur_finish<T><<<rp.n_fsh, 64, 0, s>>>(rp.probs, rp.fsh);
  }
  if (rp.n_pri) {
    Timed t(tm, K_PRIOR_APPLY, s);
    k_prior_apply<T><<<rp.n_pri, 256, 0, s>>>(rp.probs, rp.pri);
  }
  if (rp.n_pcg && one_reduction) {
    {
      Timed t(tm, K_PCG_SPMV, s);
      if (rp.pcg_rows >= kPcgRowsSparse)
        k_cg_start<T, 16><<<rp.n_pcg, 1024, 0, s>>>(rp.probs, rp.pcg);
      else
        k_cg_start<T, 4><<<rp.n_pcg, 256, 0, s>>>(rp.probs, rp.pcg);
    }
    Timed t(tm, K_PCG_CG, s, pcg_max);
    hipError_t le = hipSuccess;
    if (rp.n_probs == 1) {  // the rig view's descriptor by value
      const void *f = CgStep<T>::single(rp.pcg_rows);
      for (int it = 0; it < pcg_max && le == hipSuccess; ++it) {
        void *args[] = {(void *)&rp.single, (void *)&it};
        le = hipLaunchKernel(f, dim3(rp.n_pcg), dim3(kCgThreads), args, ubytes, s);
      }
    } else {
      const void *f = CgStep<T>::multi(rp.pcg_rows);
      for (int it = 0; it < pcg_max && le == hipSuccess; ++it) {
        void *args[] = {(void *)&rp.probs, (void *)&rp.pcg, (void *)&it};
        le = hipLaunchKernel(f, dim3(rp.n_pcg), dim3(kCgThreads), args, ubytes, s);
      }
    }
    if (le != hipSuccess) return le;
  } else {
    for (int it = 0; it < pcg_max && rp.n_pcg; ++it) {
      {
        Timed t(tm, K_PCG_SPMV, s);
        k_pcg_spmv<T><<<rp.n_pcg, 256, 0, s>>>(rp.probs, rp.pcg, it);
      }
      {
        Timed t(tm, K_PCG_UPDATE, s);
        k_pcg_update<T><<<rp.n_pcg, 256, 0, s>>>(rp.probs, rp.pcg, it);
      }
    }
  }
  // back to the cameras: rig update, recomposition, points, LM control
  if (cp.n_cam) {
    Timed t(tm, K_RIG_UPDATE, s);
    k_rig_update<T><<<cp.n_cam, 256, 0, s>>>(cp.probs, cp.cam);
  }
  if (cp.n_pt) {
    Timed t(tm, K_POINT_TRIAL, s);
    k_point_trial<T, S><<<cp.n_pt, kObsChunk, 0, s>>>(cp.probs, cp.pt);
  }
  if (cp.n_ctl) {
    Timed t(tm, K_LM_CONTROL, s);
    k_lm_control<<<cp.n_ctl, 256, 0, s>>>(cp.probs, cp.ctl);
  }
  return hipGetLastError();
}

hipError_t launch_rig_iteration(int precision, const BatchPlan &cam, const BatchPlan &rig, int pcg_max,
                                int max_tcols, hipStream_t s, KernelTimer *timer) {
  switch (precision) {
    case 0: return rig_iteration<double, double>(cam, rig, pcg_max, max_tcols, s, timer);
    case 1: return rig_iteration<float, float>(cam, rig, pcg_max, max_tcols, s, timer);
    case 2: return rig_iteration<float, _Float16>(cam, rig, pcg_max, max_tcols, s, timer);
    default: return rig_iteration<float, bf16s>(cam, rig, pcg_max, max_tcols, s, timer);
  }
}

hipError_t launch_lm_iteration(int precision, const BatchPlan &bp, int pcg_max, int max_tcols,
                               hipStream_t s, KernelTimer *timer, int part) {
  switch (precision) {
    case 0: return lm_iteration<double, double>(bp, pcg_max, max_tcols, s, timer, part);
    case 1: return lm_iteration<float, float>(bp, pcg_max, max_tcols, s, timer, part);
    case 2: return lm_iteration<float, _Float16>(bp, pcg_max, max_tcols, s, timer, part);
    default: return lm_iteration<float, bf16s>(bp, pcg_max, max_tcols, s, timer, part);
  }
}

// Test export of the stored linearisation: sqrt(w) r, sqrt(w) J_c and sqrt(w) J_p of
// every observation (internal order) from its record, rebuilt exactly as the Schur
// and back-substitution kernels rebuild them, in FP64; zeros for observations in
// fixed cameras (they have no record).  `cur`: the state the records were formed at.
template <class T, class S>
__global__ __launch_bounds__(256) void k_export_records(const ProbDev pd, int cur, double *__restrict__ r,
                                                        double *__restrict__ Jc, double *__restrict__ Jp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= pd.N) return;
  double *ro = r + 2 * (size_t)k, *jco = Jc + 12 * (size_t)k, *jpo = Jp + 6 * (size_t)k;
  const int cpos = pd.obs_rpos[k];
  if (cpos < 0) {
    for (int i = 0; i < 2; ++i) ro[i] = 0.0;
    for (int i = 0; i < 12; ++i) jco[i] = 0.0;
    for (int i = 0; i < 6; ++i) jpo[i] = 0.0;
    return;
  }
  const LinRec<T, S> &rec = ((const LinRec<T, S> *)pd.lin)[cpos];
  T f[7], R[9], J[12], P[6];
  decode(rec, f);
  load_rot(pd.pose[cur] + 12 * pd.obs_cam[k], R);
  jc_from(f, J);
  jp_from(f, R, P);
  for (int i = 0; i < 2; ++i) ro[i] = (double)rec.e[i];
  for (int i = 0; i < 12; ++i) jco[i] = (double)J[i];
  for (int i = 0; i < 6; ++i) jpo[i] = (double)P[i];
}

hipError_t launch_export_records(int precision, const ProbDev &pd, int cur, double *r, double *Jc, double *Jp,
                                 hipStream_t s) {
  if (pd.N <= 0) return hipSuccess;
  const int g = (pd.N + 255) / 256;
  switch (precision) {
    case 0: k_export_records<double, double><<<g, 256, 0, s>>>(pd, cur, r, Jc, Jp); break;
    case 1: k_export_records<float, float><<<g, 256, 0, s>>>(pd, cur, r, Jc, Jp); break;
    case 2: k_export_records<float, _Float16><<<g, 256, 0, s>>>(pd, cur, r, Jc, Jp); break;
    default: k_export_records<float, bf16s><<<g, 256, 0, s>>>(pd, cur, r, Jc, Jp); break;
  }
  return hipGetLastError();
}

hipError_t launch_eval(int precision, const BatchPlan &bp, hipStream_t s, KernelTimer *timer) {
  if (!bp.n_pt) return hipSuccess;
  Timed t(timer, K_EVAL, s);
  if (precision == 0)
    k_eval<double><<<bp.n_pt, 256, 0, s>>>(bp.probs, bp.pt);
  else
    k_eval<float><<<bp.n_pt, 256, 0, s>>>(bp.probs, bp.pt);
  return hipGetLastError();
}

// A problem's initial state restored in one launch: the pose and point buffers of index 0
// from their initial copies, and every observation active again.
__global__ __launch_bounds__(256) void k_reset(double *__restrict__ pose, const double *__restrict__ pose_init,
                                               int64_t n_pose, double *__restrict__ X,
                                               const double *__restrict__ X_init, int64_t n_X,
                                               uint32_t *__restrict__ act_words, int64_t n_words,
                                               uint8_t *__restrict__ act_tail, int n_tail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < n_pose; i += stride) pose[i] = pose_init[i];
  for (int64_t i = i0; i < n_X; i += stride) X[i] = X_init[i];
  for (int64_t i = i0; i < n_words; i += stride) act_words[i] = 0x01010101u;
  if (i0 < n_tail) act_tail[i0] = 1;
}

hipError_t launch_reset(double *pose, const double *pose_init, size_t n_pose, double *X, const double *X_init,
                        size_t n_X, uint8_t *act, size_t n_act, hipStream_t s) {
  // act: the start of a 256-byte-aligned allocation, so that its words are aligned
  const size_t n_words = n_act / 4;
  const size_t most = std::max(std::max(n_pose, n_X), n_words);
  const int grid = (int)std::max<size_t>(1, std::min<size_t>((most + 255) / 256, 2048));
  k_reset<<<grid, 256, 0, s>>>(pose, pose_init, (int64_t)n_pose, X, X_init, (int64_t)n_X, (uint32_t *)act,
                               (int64_t)n_words, act + 4 * n_words, (int)(n_act - 4 * n_words));
  return hipGetLastError();
}

hipError_t launch_cull(int precision, const BatchPlan &bp, double tau2, int method, hipStream_t s,
                       KernelTimer *timer) {
  if (!bp.n_pt) return hipSuccess;
  Timed t(timer, K_CULL, s);
  if (precision == 0)
    k_cull<double><<<bp.n_pt, 256, 0, s>>>(bp.probs, bp.pt, tau2, method);
  else
    k_cull<float><<<bp.n_pt, 256, 0, s>>>(bp.probs, bp.pt, tau2, method);
  return hipGetLastError();
}

// Triangulation from scratch, one thread per point: observations ordered by point
// (pt_start), each with its camera and normalized coordinates; a point with fewer than
// two observations, or whose triangulation fails, keeps its input value and ok = 0.
__global__ __launch_bounds__(256) void k_triangulate(int n_pts, const int32_t *__restrict__ pt_start,
                                                     const int32_t *__restrict__ cam,
                                                     const double *__restrict__ xy,
                                                     const double *__restrict__ poses, int method,
                                                     double *__restrict__ X, uint8_t *__restrict__ ok) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_pts) return;
  const int k0 = pt_start[j], n = pt_start[j + 1] - k0;
  auto get = [&](int kk, const double *&P, double &x, double &y) {
    const int k = k0 + kk;
    P = poses + 12 * (size_t)cam[k];
    x = xy[2 * (size_t)k];
    y = xy[2 * (size_t)k + 1];
    return true;
  };
  double Xn[3];
  const bool good = n >= 2 && (method == 1 ? tri_dlt(n, get, Xn) : tri_midpoint(n, get, Xn));
  if (good) {
    X[3 * (size_t)j] = Xn[0];
    X[3 * (size_t)j + 1] = Xn[1];
    X[3 * (size_t)j + 2] = Xn[2];
  }
  ok[j] = good ? 1 : 0;
}

// RANSAC triangulation per track, one thread per point: hypothesis h = 0 .. n_hyp - 1
// takes the observation pair a = h mod n, b = (a + 1 + (h div n) mod (n - 1)) mod n (every
// ordered pair once within n (n - 1) hypotheses), triangulates it by the two-ray
// midpoint and counts the track's observations in front of their camera with a
// reprojection error of at most sqrt(tau2) pixels; the first hypothesis with the most
// inliers wins, and with at least two inliers the point is triangulated from them
// (midpoint or DLT).  inl[k] flags the inliers (all 0 when the track fails).
__global__ __launch_bounds__(256) void k_triangulate_ransac(int n_pts, const int32_t *__restrict__ pt_start,
                                                            const int32_t *__restrict__ cam,
                                                            const double *__restrict__ xy,
                                                            const double *__restrict__ poses,
                                                            const double *__restrict__ Kc, double tau2,
                                                            int n_hyp, int method, double *__restrict__ X,
                                                            uint8_t *__restrict__ ok, uint8_t *__restrict__ inl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_pts) return;
  const int k0 = pt_start[j], n = pt_start[j + 1] - k0;
  auto give_up = [&]() {
    ok[j] = 0;
    for (int k = 0; k < n; ++k) inl[k0 + k] = 0;
  };
  if (n < 2) {
    give_up();
    return;
  }
  auto obs = [&](int kk, const double *&P, double &x, double &y) {
    const int k = k0 + kk;
    P = poses + 12 * (size_t)cam[k];
    x = xy[2 * (size_t)k];
    y = xy[2 * (size_t)k + 1];
  };
  auto is_inlier = [&](int kk, const double Xp[3]) {
    const double *P;
    double x, y;
    obs(kk, P, x, y);
    const double pz = P[6] * Xp[0] + P[7] * Xp[1] + P[8] * Xp[2] + P[11];
    if (!(pz > kZMin)) return false;
    const double px = P[0] * Xp[0] + P[1] * Xp[1] + P[2] * Xp[2] + P[9];
    const double py = P[3] * Xp[0] + P[4] * Xp[1] + P[5] * Xp[2] + P[10];
    const double *K = Kc + 4 * (size_t)cam[k0 + kk];
    const double r0 = K[0] * (px / pz - x), r1 = K[1] * (py / pz - y);
    return r0 * r0 + r1 * r1 <= tau2;
  };
  auto pair_point = [&](int h, double Xp[3]) {
    const int a = h % n, b = (a + 1 + (h / n) % (n - 1)) % n;
    auto get = [&](int kk, const double *&P, double &x, double &y) {
      if (kk != a && kk != b) return false;
      obs(kk, P, x, y);
      return true;
    };
    return tri_midpoint(n, get, Xp);
  };
  int best = -1, best_h = -1;
  for (int h = 0; h < n_hyp; ++h) {
    double Xp[3];
    if (!pair_point(h, Xp)) continue;
    int cnt = 0;
    for (int kk = 0; kk < n; ++kk) cnt += is_inlier(kk, Xp) ? 1 : 0;
    if (cnt > best) {
      best = cnt;
      best_h = h;
    }
  }
  if (best < 2) {
    give_up();
    return;
  }
  double Xb[3];
  pair_point(best_h, Xb);
  for (int kk = 0; kk < n; ++kk) inl[k0 + kk] = is_inlier(kk, Xb) ? 1 : 0;
  auto get_in = [&](int kk, const double *&P, double &x, double &y) {
    if (!inl[k0 + kk]) return false;
    obs(kk, P, x, y);
    return true;
  };
  double Xn[3];
  const bool good = method == 1 ? tri_dlt(n, get_in, Xn) : tri_midpoint(n, get_in, Xn);
  if (!good) {
    give_up();
    return;
  }
  X[3 * (size_t)j] = Xn[0];
  X[3 * (size_t)j + 1] = Xn[1];
  X[3 * (size_t)j + 2] = Xn[2];
  ok[j] = 1;
}

hipError_t launch_triangulate_ransac(int n_pts, const int32_t *pt_start, const int32_t *cam, const double *xy,
                                     const double *poses, const double *Kc, double tau2, int n_hyp, int method,
                                     double *X, uint8_t *ok, uint8_t *inl, hipStream_t s) {
  if (n_pts <= 0) return hipSuccess;
  k_triangulate_ransac<<<(n_pts + 255) / 256, 256, 0, s>>>(n_pts, pt_start, cam, xy, poses, Kc, tau2, n_hyp,
                                                           method, X, ok, inl);
  return hipGetLastError();
}

hipError_t launch_triangulate(int n_pts, const int32_t *pt_start, const int32_t *cam, const double *xy,
                              const double *poses, int method, double *X, uint8_t *ok, hipStream_t s) {
  if (n_pts <= 0) return hipSuccess;
  k_triangulate<<<(n_pts + 255) / 256, 256, 0, s>>>(n_pts, pt_start, cam, xy, poses, method, X, ok);
  return hipGetLastError();
}

hipError_t launch_pose_gn(int n_req, PoseDev *reqs, const double *X, const float *uv, hipStream_t s,
                          KernelTimer *timer) {
  if (n_req <= 0) return hipSuccess;
  Timed t(timer, K_POSE_GN, s);
  k_pose_gn<<<n_req, kPoseThreads, 0, s>>>(reqs, X, uv);
  return hipGetLastError();
}

}  // namespace bax
