// Device-side track model for the gfx950 kernels: helix transport, Kalman update,
// sector rotation and the merge chi2, in FP32.
//
// Bit-exactness contract: every expression below is evaluated in exactly the
// order written (the library is compiled with -ffp-contract=off and without
// fast-math, so no FMA contraction and no reassociation), with IEEE
// round-to-nearest +, -, *, / and sqrt.  The CPU oracle follows the same
// written formulas; parity tests compare the two bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace tpc {

constexpr int kRows = 152;
constexpr int kSectors = 36;
constexpr int kHalf = 18;
constexpr int kSlotsPerJob = kSectors * kRows;

// Geometry and derived FP32 constants, formed on the host in double and rounded once.
struct Consts {
  float x[kRows];        // pad-row planes: 85 + r*160/151 cm
  float cb;              // -kappa*B: signed curvature per unit q/pT (1/cm per 1/GeV)
  float cos20, sin20, tan10;
  float vy, vz;          // sigma^2
  float cut2;            // link_cut^2
  float cut2_above;      // the float just above cut2 (cut2 is a normal float)
  float smax;
  float win_dy_slope, win_dy_const, win_dz_slope, win_dz_const, link_cut;
  float nwin, chi2_follow;
  int32_t max_miss, min_hits;
  float prior0[5], prior1[5];
  float merge_edge, chi2_merge, merge_dz;
  float v_drift;         // cm/us
  int membrane;          // 1: merge across the central membrane
};

// lower-triangle index of a symmetric 5x5 (i >= j)
__host__ __device__ constexpr int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// Correctly rounded FP32 square root and division.  llvm.sqrt.f32 and fdiv are
// lowered to correctly rounded sequences under HIP's default
// -fhip-fp32-correctly-rounded-divide-sqrt (HIP's __fsqrt_rn is the approximate
// native instruction unless OCML_BASIC_ROUNDED_OPERATIONS is defined).
__device__ __forceinline__ float sqrt_rn(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ float div_rn(float a, float b) { return a / b; }

// (hi, lo) += d with an exact two-sum; hi stays fl(hi + lo).
__device__ __forceinline__ void acc(float& hi, float& lo, float d) {
  const float s = hi + d;
  const float bb = s - hi;
  const float e = (hi - (s - bb)) + (d - bb);
  const float t = lo + e;
  hi = s + t;
  lo = t - (hi - s);
}

__device__ __forceinline__ bool finite_f(float v) { return v - v == 0.f; }

// asin(u)/u and its derivative over u: Taylor coefficients of asin (Horner in w = u^2)
// for |u| <= 1/2; for larger |u| the identity asin(u) = pi/2 - 2 asin(sqrt((1-|u|)/2)).
__device__ __forceinline__ float series_A(float w) {
  float a = 0x1.3fde50p-7f;
  a = 0x1.7a8788p-7f + w * a;
  a = 0x1.c9999ap-7f + w * a;
  a = 0x1.1c4ec4p-6f + w * a;
  a = 0x1.6e8ba2p-6f + w * a;
  a = 0x1.f1c71cp-6f + w * a;
  a = 0x1.6db6dcp-5f + w * a;
  a = 0x1.333334p-4f + w * a;
  a = 0x1.555556p-3f + w * a;
  a = 0x1p+0f + w * a;
  return a;
}
__device__ __forceinline__ float series_B(float w) {
  float b = 0x1.3ce4aep-3f;
  b = 0x1.497922p-3f + w * b;
  b = 0x1.57ab0cp-3f + w * b;
  b = 0x1.67da1ap-3f + w * b;
  b = 0x1.7a8788p-3f + w * b;
  b = 0x1.906666p-3f + w * b;
  b = 0x1.aa7628p-3f + w * b;
  b = 0x1.ca2e8cp-3f + w * b;
  b = 0x1.f1c71cp-3f + w * b;
  b = 0x1.124924p-2f + w * b;
  b = 0x1.333334p-2f + w * b;
  b = 0x1.555556p-2f + w * b;
  return b;
}
__device__ __forceinline__ void asinc(float u, float& A, float& B) {
  const float au = fabsf(u);
  const float w = u * u;
  if (au <= 0.5f) {
    A = series_A(w);
    B = series_B(w);
  } else {
    const float v = sqrt_rn((1.0f - au) * 0.5f);
    const float asn = 0x1.921fb6p+0f - 2.0f * (v * series_A(v * v));
    A = div_rn(asn, au);
    const float g = div_rn(1.0f, sqrt_rn((1.0f - u) * (1.0f + u)));
    B = div_rn(g - A, w);
  }
}

struct State {
  float P[5];   // y, z, sin(phi), tan(lambda), q/pT  (hi parts)
  float L[5];   // compensation (lo parts)
  float C[15];  // covariance, lower triangle
};

// Helix transport from plane x1 to plane x2 on the cos(phi) > 0 branch with the
// analytic Jacobian J and C' = J C J^T.  On failure the state is untouched.
__device__ __forceinline__ bool propagate(State& S, float x1, float x2, const Consts& k) {
  const float dx = x2 - x1;
  if (dx == 0.f) return true;
  const float cb = k.cb;
  const float curv = S.P[4] * cb;
  const float s1 = S.P[2];
  const float s2 = s1 + curv * dx;
  if (!(fabsf(s2) < k.smax)) return false;
  const float c1 = sqrt_rn((1.f - s1) * (1.f + s1));
  const float c2 = sqrt_rn((1.f - s2) * (1.f + s2));
  const float cc = c1 + c2;
  const float f = div_rn(s1 + s2, cc);
  const float dy = dx * f;
  float ch = sqrt_rn(dx * dx + dy * dy);
  if (dx < 0.f) ch = -ch;
  const float u = curv * ch * 0.5f;
  if (!(fabsf(u) < 1.f)) return false;
  float A, B;
  asinc(u, A, B);
  const float g = div_rn(1.f, sqrt_rn((1.f - u) * (1.f + u)));
  const float dS = ch * A;
  const float q1 = div_rn(s1, c1);
  const float q2 = div_rn(s2, c2);
  const float fs = div_rn(2.f + f * (q1 + q2), cc);
  const float fc = div_rn(dx * (1.f + f * q2), cc);
  const float ja = dx * fs;
  const float jb = dx * fc * cb;
  const float chs = div_rn(dy * ja, ch);
  const float chk = div_rn(dy * jb, ch);
  const float dSs = g * chs;
  const float dSk = g * chk + ch * ch * u * B * 0.5f * cb;
  const float t = S.P[3];
  const float je = t * dSs;
  const float jf = dS;
  const float jg = t * dSk;
  const float jh = cb * dx;
  acc(S.P[0], S.L[0], dy);
  acc(S.P[1], S.L[1], t * dS);
  acc(S.P[2], S.L[2], curv * dx);
  float c[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) c[i][j] = S.C[tri(i, j)];
  float M[5][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    M[0][j] = c[0][j] + ja * c[2][j] + jb * c[4][j];
    M[1][j] = c[1][j] + je * c[2][j] + jf * c[3][j] + jg * c[4][j];
    M[2][j] = c[2][j] + jh * c[4][j];
    M[3][j] = c[3][j];
    M[4][j] = c[4][j];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float n0 = M[i][0] + ja * M[i][2] + jb * M[i][4];
    const float n1 = M[i][1] + je * M[i][2] + jf * M[i][3] + jg * M[i][4];
    const float n2 = M[i][2] + jh * M[i][4];
    const float n[5] = {n0, n1, n2, M[i][3], M[i][4]};
#pragma unroll
    for (int j = 0; j <= i; ++j) S.C[tri(i, j)] = n[j];
  }
  return true;
}

// Inverse of the innovation covariance S = C[0:2,0:2] + diag(vy, vz).
struct SInv {
  float i00, i10, i11;
  bool ok;
};
__device__ __forceinline__ SInv s_inverse(const float* C, float vy, float vz) {
  SInv r;
  const float S00 = C[0] + vy;
  const float S10 = C[1];
  const float S11 = C[2] + vz;
  const float det = S00 * S11 - S10 * S10;
  r.ok = det > 0.f;
  const float idet = div_rn(1.f, det);
  r.i00 = S11 * idet;
  r.i10 = -(S10 * idet);
  r.i11 = S00 * idet;
  return r;
}
__device__ __forceinline__ float chi2_of(const SInv& s, float r0, float r1) {
  const float a0 = s.i00 * r0 + s.i10 * r1;
  const float a1 = s.i10 * r0 + s.i11 * r1;
  return r0 * a0 + r1 * a1;
}

// Kalman update with the cluster (my, mz).  Measured rows/columns: C'(i,m) = K(i,m) V;
// the rest C - K H C.  On failure the state is untouched.
__device__ __forceinline__ bool kf_update(State& S, float my, float mz, const Consts& k, float* chi2_out) {
  const SInv si = s_inverse(S.C, k.vy, k.vz);
  if (!si.ok) return false;
  const float r0 = (my - S.P[0]) - S.L[0];
  const float r1 = (mz - S.P[1]) - S.L[1];
  const float chi2 = chi2_of(si, r0, r1);
  float c0[5], c1[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    c0[i] = S.C[tri(i, 0)];
    c1[i] = S.C[tri(i, 1)];
  }
  float K0[5], K1[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    K0[i] = c0[i] * si.i00 + c1[i] * si.i10;
    K1[i] = c0[i] * si.i10 + c1[i] * si.i11;
  }
  float Pn[5], Ln[5], Cn[15];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    Pn[i] = S.P[i];
    Ln[i] = S.L[i];
    acc(Pn[i], Ln[i], K0[i] * r0 + K1[i] * r1);
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    Cn[tri(i, 0)] = K0[i] * k.vy;
    if (i >= 1) Cn[tri(i, 1)] = K1[i] * k.vz;
#pragma unroll
    for (int j = 2; j <= i; ++j) Cn[tri(i, j)] = S.C[tri(i, j)] - (K0[i] * c0[j] + K1[i] * c1[j]);
  }
  bool fin = true;
#pragma unroll
  for (int i = 0; i < 5; ++i) fin = fin && finite_f(Pn[i]);
#pragma unroll
  for (int i = 0; i < 15; ++i) fin = fin && finite_f(Cn[i]);
  if (!fin) return false;
  if (!(fabsf(Pn[2]) < k.smax)) return false;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    S.P[i] = Pn[i];
    S.L[i] = Ln[i];
  }
#pragma unroll
  for (int i = 0; i < 15; ++i) S.C[i] = Cn[i];
  if (chi2_out) *chi2_out = chi2;
  return true;
}

// Re-express the state in the frame of the adjacent sector `to` (same side; the
// sector angle changes by d = +-20 deg).  x is updated to the rotated plane.
// Covariance by the first-order Jacobian of "rotate, then move along the helix
// back to the rotated plane": dy'/dy = c/c', dz'/dy = -t sin d / c',
// ds'/dy = -k cb sin d (the direction turns while moving back), ds'/ds = c'/c.
__device__ __forceinline__ bool rotate(State& S, float& x, int from, int to, const Consts& k) {
  const int df = ((to % kHalf) - (from % kHalf) + kHalf) % kHalf;
  if (df != 1 && df != kHalf - 1) return false;
  const float ca = k.cos20;
  const float sa = df == 1 ? k.sin20 : -k.sin20;
  const float s = S.P[2];
  const float c = sqrt_rn((1.f - s) * (1.f + s));
  const float xn = x * ca + S.P[0] * sa;
  const float yn = S.P[0] * ca - x * sa;
  const float sn = s * ca - c * sa;
  const float cn = c * ca + s * sa;
  if (!(cn > 0.f) || !(fabsf(sn) < k.smax)) return false;
  const float ja = div_rn(c, cn);
  const float jb = -div_rn(S.P[3] * sa, cn);
  const float jc = -(S.P[4] * k.cb * sa);
  const float je = div_rn(cn, c);
  float c5[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) c5[i][j] = S.C[tri(i, j)];
  float M[5][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    M[0][j] = ja * c5[0][j];
    M[1][j] = jb * c5[0][j] + c5[1][j];
    M[2][j] = jc * c5[0][j] + je * c5[2][j];
    M[3][j] = c5[3][j];
    M[4][j] = c5[4][j];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float n[5] = {ja * M[i][0], jb * M[i][0] + M[i][1], jc * M[i][0] + je * M[i][2], M[i][3], M[i][4]};
#pragma unroll
    for (int j = 0; j <= i; ++j) S.C[tri(i, j)] = n[j];
  }
  S.P[0] = yn;
  S.P[2] = sn;
  S.L[0] = 0.f;
  S.L[2] = 0.f;
  x = xn;
  bool fin = true;
#pragma unroll
  for (int i = 0; i < 5; ++i) fin = fin && finite_f(S.P[i]);
#pragma unroll
  for (int i = 0; i < 15; ++i) fin = fin && finite_f(S.C[i]);
  return fin;
}

// ---- track-model compression: the predicted position of a cluster on a fitted track
// (the state parts of rotate() and propagate(), same operations in the same order).

// One sector turn of the state (y, z, sin phi, tan lambda, q/pT) at plane x; same side only.
__device__ __forceinline__ bool rotate_state(float* P, float& x, int from, int to, const Consts& k) {
  if (from / kHalf != to / kHalf) return false;
  const int df = ((to % kHalf) - (from % kHalf) + kHalf) % kHalf;
  if (df != 1 && df != kHalf - 1) return false;
  const float ca = k.cos20;
  const float sa = df == 1 ? k.sin20 : -k.sin20;
  const float s = P[2];
  const float c = sqrt_rn((1.f - s) * (1.f + s));
  const float xn = x * ca + P[0] * sa;
  const float yn = P[0] * ca - x * sa;
  const float sn = s * ca - c * sa;
  const float cn = c * ca + s * sa;
  if (!(cn > 0.f) || !(fabsf(sn) < k.smax)) return false;
  P[0] = yn;
  P[2] = sn;
  x = xn;
  bool fin = true;
#pragma unroll
  for (int i = 0; i < 5; ++i) fin = fin && finite_f(P[i]);
  return fin;
}

// Helix transport of the state alone from plane x1 to plane x2.
__device__ __forceinline__ bool transport_state(float* P, float x1, float x2, const Consts& k) {
  const float dx = x2 - x1;
  if (dx == 0.f) return true;
  const float curv = P[4] * k.cb;
  const float s1 = P[2];
  const float s2 = s1 + curv * dx;
  if (!(fabsf(s2) < k.smax)) return false;
  const float c1 = sqrt_rn((1.f - s1) * (1.f + s1));
  const float c2 = sqrt_rn((1.f - s2) * (1.f + s2));
  const float f = div_rn(s1 + s2, c1 + c2);
  const float dy = dx * f;
  float ch = sqrt_rn(dx * dx + dy * dy);
  if (dx < 0.f) ch = -ch;
  const float u = curv * ch * 0.5f;
  if (!(fabsf(u) < 1.f)) return false;
  float A, B;
  asinc(u, A, B);
  P[0] = P[0] + dy;
  P[1] = P[1] + P[3] * (ch * A);
  P[2] = P[2] + curv * dx;
  return true;
}

// Collision time of a track fitted to state Pf at plane xref of sector `sector`: the
// state transported to the beam line (x = 0), where a primary's measured z is the drift
// shift of its collision time, -v_d t0 on side A and +v_d t0 on side C.
__device__ __forceinline__ float collision_time(const float* Pf, float xref, int sector, const Consts& k) {
  float P[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) P[i] = Pf[i];
  if (!transport_state(P, xref, 0.f, k)) return __builtin_nanf("");
  const float z0 = P[1];
  return div_rn(sector < kHalf ? -z0 : z0, k.v_drift);
}

// Predicted (y, z) at pad row `row` of sector `sec` for a track fitted to state Pf at plane
// xref in the frame of sector sref: the state is turned one sector at a time towards `sec`
// (the shorter way round, same side of the membrane), then transported to the row's plane.
__device__ __forceinline__ bool predict_yz(const float* Pf, float xref, int sref, int sec, int row,
                                           const Consts& k, float& py, float& pz) {
  if (sref < 0 || sref >= kSectors || sec / kHalf != sref / kHalf) return false;
  float P[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) P[i] = Pf[i];
  float x = xref;
  const int steps = ((sec % kHalf) - (sref % kHalf) + kHalf) % kHalf;
  const int dir = steps <= kHalf / 2 ? 1 : -1;
  const int nst = dir == 1 ? steps : kHalf - steps;
  int cur = sref;
  for (int i = 0; i < nst; ++i) {
    const int nxt = (cur / kHalf) * kHalf + (cur % kHalf + dir + kHalf) % kHalf;
    if (!rotate_state(P, x, cur, nxt, k)) return false;
    cur = nxt;
  }
  if (!transport_state(P, x, k.x[row], k)) return false;
  py = P[0];
  pz = P[1];
  return true;
}

// chi2 = d^T (CA + CB)^-1 d by a 5x5 Cholesky factorisation in fixed order.
// The same over y, sin phi, tan lambda and q/pT (indices 0, 2, 3, 4): the comparison across
// the central membrane, where z is off by the drift of the collision time.
__device__ __forceinline__ float membrane_chi2(const float* PA, const float* CA, const float* PB,
                                               const float* CB) {
  constexpr int ix[4] = {0, 2, 3, 4};
  float S[10], d[4], L[10];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) S[tri(i, j)] = CA[tri(ix[i], ix[j])] + CB[tri(ix[i], ix[j])];
#pragma unroll
  for (int i = 0; i < 4; ++i) d[i] = PA[ix[i]] - PB[ix[i]];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float a = S[tri(i, j)];
#pragma unroll
      for (int q = 0; q < j; ++q) a = a - L[tri(i, q)] * L[tri(j, q)];
      if (i == j) {
        if (!(a > 0.f)) return __builtin_inff();
        L[tri(i, i)] = sqrt_rn(a);
      } else {
        L[tri(i, j)] = div_rn(a, L[tri(j, j)]);
      }
    }
  }
  float w[4];
  float c = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float a = d[i];
#pragma unroll
    for (int q = 0; q < i; ++q) a = a - L[tri(i, q)] * w[q];
    w[i] = div_rn(a, L[tri(i, i)]);
    c = c + w[i] * w[i];
  }
  return c;
}

// Collision time of a membrane link from the two pieces' z at the same plane: side A
// measures z - v t0, side C z + v t0.
__device__ __forceinline__ float membrane_t0(bool a_side, float za, float zb, const Consts& k) {
  return a_side ? div_rn(zb - za, 2.0f * k.v_drift) : div_rn(za - zb, 2.0f * k.v_drift);
}

__device__ __forceinline__ float merge_chi2(const float* PA, const float* CA, const float* PB,
                                            const float* CB) {
  float S[15], d[5], L[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) S[i] = CA[i] + CB[i];
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = PA[i] - PB[i];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float a = S[tri(i, j)];
#pragma unroll
      for (int q = 0; q < j; ++q) a = a - L[tri(i, q)] * L[tri(j, q)];
      if (i == j) {
        if (!(a > 0.f)) return __builtin_inff();
        L[tri(i, i)] = sqrt_rn(a);
      } else {
        L[tri(i, j)] = div_rn(a, L[tri(j, j)]);
      }
    }
  }
  float w[5];
  float c = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float a = d[i];
#pragma unroll
    for (int q = 0; q < i; ++q) a = a - L[tri(i, q)] * w[q];
    w[i] = div_rn(a, L[tri(i, i)]);
    c = c + w[i] * w[i];
  }
  return c;
}

}  // namespace tpc
