// Forward-mode "jets" for the forward Laplacian (Methods, efficient
// Laplacian, eqs. forward_lap_jac and forward_lap_lap): a value, its
// gradient along ND input directions and its Laplacian summed over them.
#pragma once
#include "common.hpp"

namespace fire {

template <typename T> struct J3 {
  T v, g[3], l;
};

template <typename T> FIRE_DEV J3<T> jconst(T c) { return J3<T>{c, {T(0), T(0), T(0)}, T(0)}; }
template <typename T> FIRE_DEV J3<T> jadd(const J3<T>& a, const J3<T>& b) {
  return J3<T>{a.v + b.v, {a.g[0] + b.g[0], a.g[1] + b.g[1], a.g[2] + b.g[2]}, a.l + b.l};
}
template <typename T> FIRE_DEV void jaxpy(J3<T>& y, T a, const J3<T>& x) {
  y.v += a * x.v; y.g[0] += a * x.g[0]; y.g[1] += a * x.g[1]; y.g[2] += a * x.g[2]; y.l += a * x.l;
}
// product rule: (ab)' = a b' + b a';  Lap(ab) = a Lap b + b Lap a + 2 grad a . grad b
template <typename T> FIRE_DEV J3<T> jmul(const J3<T>& a, const J3<T>& b) {
  J3<T> r;
  r.v = a.v * b.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.v * b.g[k] + b.v * a.g[k];
  r.l = a.v * b.l + b.v * a.l + T(2) * (a.g[0] * b.g[0] + a.g[1] * b.g[1] + a.g[2] * b.g[2]);
  return r;
}
// chain rule for a scalar function with value f, derivatives f1, f2 at x.v
template <typename T> FIRE_DEV J3<T> jchain(const J3<T>& x, T f, T f1, T f2) {
  J3<T> r;
  r.v = f;
  for (int k = 0; k < 3; ++k) r.g[k] = f1 * x.g[k];
  r.l = f1 * x.l + f2 * (x.g[0] * x.g[0] + x.g[1] * x.g[1] + x.g[2] * x.g[2]);
  return r;
}
template <typename T> FIRE_DEV J3<T> jsilu(const J3<T>& x) {
  T f, f1, f2;
  silu3(x.v, f, f1, f2);
  return jchain(x, f, f1, f2);
}

// Jets of the pair features w.r.t. the displacement d = r_a - r_b (3 dirs):
//   out[0..4)   rescaled features log(1+r)/r * [r, dx, dy, dz]
//   out[4..4+h2) second filter hidden layer
//   out[12..44) radial part f_cut(r/c) exp(-sigma_k^2 r^2)
// Each jet occupies 5 consecutive T (v, gx, gy, gz, l); out[44*5] holds f_cut.
constexpr int JFEAT = 44 * 5 + 4;

// W2 entry (j, k) is read at W2[j s2j + k s2k]: (h2, 1) for the row-major
// parameter, (1, kMaxH1) for a transposed copy staged in LDS.
template <typename T>
FIRE_DEV void pair_feature_jets(T dx, T dy, T dz, const T* W1, const T* b1, const T* W2, int s2j, int s2k,
                                const T* b2, const T* sig, T cut, const Dims& D, T* out) {
  T r = sqrt(dx * dx + dy * dy + dz * dz);
  J3<T> rj;
  rj.v = r;
  if (r > T(0)) {
    T ir = T(1) / r;
    rj.g[0] = dx * ir; rj.g[1] = dy * ir; rj.g[2] = dz * ir;
    rj.l = T(2) * ir;
  } else {
    rj.g[0] = rj.g[1] = rj.g[2] = T(0);
    rj.l = T(0);
  }
  J3<T> e4[4];
  e4[0] = rj;
  e4[1] = J3<T>{dx, {T(1), T(0), T(0)}, T(0)};
  e4[2] = J3<T>{dy, {T(0), T(1), T(0)}, T(0)};
  e4[3] = J3<T>{dz, {T(0), T(0), T(1)}, T(0)};
  T f, f1, f2;
  log1p_over3(r, f, f1, f2);
  J3<T> lo = jchain(rj, f, f1, f2);
  auto put = [&](int slot, const J3<T>& j) {
    T* o = out + 5 * slot;
    o[0] = j.v; o[1] = j.g[0]; o[2] = j.g[1]; o[3] = j.g[2]; o[4] = j.l;
  };
  for (int k = 0; k < 4; ++k) put(k, jmul(lo, e4[k]));
  J3<T> z1[kMaxH1];
  for (int k = 0; k < D.h1; ++k) {
    J3<T> a = jconst(b1[k]);
    for (int j = 0; j < 4; ++j) jaxpy(a, W1[j * D.h1 + k], e4[j]);
    z1[k] = jsilu(a);
  }
  for (int k = 0; k < D.h2; ++k) {
    J3<T> a = jconst(b2[k]);
    for (int j = 0; j < D.h1; ++j) jaxpy(a, W2[j * s2j + k * s2k], z1[j]);
    put(4 + k, jsilu(a));
  }
  fcut3(r / cut, f, f1, f2);
  J3<T> fc = jchain(rj, f, f1 / cut, f2 / (cut * cut));
  for (int k = 0; k < D.G; ++k) {
    T a = sig[k] * sig[k];
    T ex = exp(-a * r * r);
    J3<T> gk = jchain(rj, ex, T(-2) * a * r * ex, (T(4) * a * a * r * r - T(2) * a) * ex);
    put(12 + k, jmul(fc, gk));
  }
  out[44 * 5] = f;
}

template <typename T>
FIRE_DEV void pair_feature_jets(T dx, T dy, T dz, const T* W1, const T* b1, const T* W2, const T* b2, const T* sig,
                                T cut, const Dims& D, T* out) {
  pair_feature_jets<T>(dx, dy, dz, W1, b1, W2, D.h2, 1, b2, sig, cut, D, out);
}

template <typename T> FIRE_DEV J3<T> jload(const T* p) { return J3<T>{p[0], {p[1], p[2], p[3]}, p[4]}; }

}  // namespace fire
