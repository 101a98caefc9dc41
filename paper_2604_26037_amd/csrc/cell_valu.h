// Cell operators on the vector ALUs: the implementation shared by the
// translation units that instantiate it (kernels_cell_valu.hip: K + V on
// cells of one size; kernels_cell_gen_f32.hip / _f64.hip: per-cell geometry,
// the GGA term and the mass term; kernels_cell_step.hip /
// kernels_cell_step_gen.hip: the filter's fused Chebyshev step).
//
// Local (cell) part of the Hamiltonian on the vector ALUs:
// Y += alpha (K + V [+ GGA]) X over the cells of one colour (eq. "FEM Ham
// entries", applied cell by cell as in the operator-action subsection),
// sum-factorized along the three axes of each hexahedral cell.
//
// Why not the matrix cores here: in FP32 the gfx950 matrix cores deliver the
// same rate per SIMD as non-packed FP32 FMAs would at 2x (157 vs 79 TFLOP/s),
// but every 1-D contraction of a degree-6 element has only 7 or 8 outputs,
// so a 16x16x4 FP32 MFMA leaves half of its outputs in padding and the
// padded contractions cost 2.2x the useful work.  Written as plain FMAs on
// lines of 7-8 values, each 1-D operator can also use the reflection
// symmetry of the GLL nodes and Gauss points (l_a(-x) = l_{p-a}(x)): with
// e_a = x_a + x_{p-a} and o_a = x_a - x_{p-a} a 7 -> 8 contraction becomes a
// 4x4 and a 4x3 product plus 8 additions (42 operations instead of 56 FMAs),
// and the symmetric, centro-symmetric 1-D stiffness and mass tables a 4x4
// and a 3x3 product.  The 1-D tables (Lagrange values of the GLL basis at the
// Gauss points, reference stiffness and mass) depend only on the degree, so
// they are compile-time constants of the kernel: every coefficient is an
// instruction literal and no table is read at run time.
//
// One workgroup handles one (cell, column tile) item at a time: FP32 8
// columns and 512 threads, FP64 4 columns and 256 threads; thread t owns
// column t % CB and line t / CB (of at most 64) of each pass.  Data of the item live in three LDS slabs with the column
// fastest and the x index padded to 9 (so the 8 lines of a wave start 8
// banks apart along every axis: no bank conflicts beyond the two cycles a
// 64-lane access needs):
//   U: the gathered cell values, then the V path in place (up to 8^3),
//   K, M: the x-contractions K1 U and M1 U, then the kinetic y and z passes.
// Passes:
//   P1 x: U -> B U (in place, 7 -> 8), K1 U -> K, M1 U -> M
//   P2 y: B (U)   P3 z: B, times V(q) W_q   P4 z: B^T   P5 y: B^T
//   (P3 and P4 run on the same lines, so one thread takes its line through
//   both in registers, with no barrier between them)
//   P6 x: B^T -> U (the V term, 7^3)
//   P7 y: K <- fx M1 K + fy K1 M,  M <- M1 M
//   P8 z: K <- U + M1 K + fz K1 M  (the cell result)
// then the colour-ordered read-modify-write of the result into Y.  The next
// item's gathered values and this item's old output rows are loaded into
// registers while the passes run, as in the matrix-core kernel.
//
// General operators (graded meshes: every cell a box of its own size; the
// GGA term) use variants of the same kernel:
//   - per-cell geometry: fx, fy, fz and det J of the item's cell from a
//     per-cell table (V(q) W_q already carries the cell's det J);
//   - the GGA term (eq. "FEM Ham entries"): with u the field at the Gauss
//     points and v_d = W_q det J (2/h_d) V_GGA,d, the cell adds
//     B^T [sum_d v_d (D_d u) + D_d^T (v_d u)], D_d the collocation derivative
//     through the Gauss points along axis d.  P3 keeps u in U and writes
//     V u plus the z part to a fourth slab G; two more passes add the y and x
//     parts; P4 reads G;
//   - the mass term det J_e M (the S apply and the -lambda M part of the
//     residual): P1 (M1 only), P7 (M1 only) and P8 (M1 only).
//
// The filter's step (Algorithm 2, step 4) runs as the step variants: the
// input-side 1-D tables have their columns divided by the GLL weights
// (doubled on the end nodes), which applies det J M_D^{-1} to the gathered
// R_Y' on the way in, so the block T = M_D^{-1} R_Y' is never stored (on
// graded meshes a node on a face whose neighbour has another size is
// scaled by the ratio of the two lumped masses when it is staged); and the
// cell making the first visit of a DOF in the colour order first replaces
// the old value by the node part of the step, -a c R_Y' - zeta zeta' R_X +
// a lambda_n Y.

#pragma once

#include <type_traits>
#include <utility>

#include "kernels.h"

namespace pawfe {

namespace {

// ---- compile-time reference-element tables -----------------------------------

namespace ref1d {

constexpr double kPi = 3.14159265358979323846;

// cos on [0, pi] by its Taylor series about 0 (after folding to [0, pi/2])
constexpr double cos_c(double x) {
  bool neg = false;
  if (x > kPi / 2) {
    x = kPi - x;
    neg = true;
  }
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return neg ? -sum : sum;
}

constexpr double abs_c(double x) { return x < 0 ? -x : x; }

// P_n(x), P_n'(x), P_n''(x) by the three-term recurrence and the Legendre ODE
struct Leg {
  double P, dP, d2P;
};
constexpr Leg legendre(int n, double x) {
  double p0 = 1.0, p1 = x;
  if (n == 0) return {1.0, 0.0, 0.0};
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  // p1 = P_n, p0 = P_{n-1}
  const double dP = n * (x * p1 - p0) / (x * x - 1.0);
  const double d2P = (2.0 * x * dP - n * (n + 1.0) * p1) / (1.0 - x * x);
  return {p1, dP, d2P};
}

// P_n(x) alone (also at x = +-1)
constexpr double legendre_P(int n, double x) {
  double p0 = 1.0, p1 = x;
  if (n == 0) return 1.0;
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  return p1;
}

template <int N>
struct Rule {
  double x[N] = {};
  double w[N] = {};
};

// N-point Gauss-Legendre rule, ascending nodes
template <int N>
constexpr Rule<N> gauss() {
  Rule<N> r{};
  for (int i = 0; i < N; ++i) {
    double xi = -cos_c(kPi * (i + 0.75) / (N + 0.5));
    for (int it = 0; it < 60; ++it) {
      const Leg l = legendre(N, xi);
      const double dx = l.P / l.dP;
      xi -= dx;
      if (abs_c(dx) < 1e-17) break;
    }
    const Leg l = legendre(N, xi);
    r.x[i] = xi;
    r.w[i] = 2.0 / ((1.0 - xi * xi) * l.dP * l.dP);
  }
  return r;
}

// GLL nodes of degree P (P + 1 points, ascending): -1, the roots of P_P', +1
template <int P>
constexpr Rule<P + 1> gll() {
  Rule<P + 1> r{};
  r.x[0] = -1.0;
  r.x[P] = 1.0;
  for (int j = 1; j < P; ++j) {
    double xj = -cos_c(kPi * j / P);
    for (int it = 0; it < 60; ++it) {
      const Leg l = legendre(P, xj);
      const double dx = l.dP / l.d2P;
      xj -= dx;
      if (abs_c(dx) < 1e-17) break;
    }
    r.x[j] = xj;
  }
  return r;
}

// Even-odd form of the 1-D tables of degree NP - 1 with NQ Gauss points.
//   B[q][a] = l_a(eta_q)   (Lagrange basis through the GLL nodes)
//   K[a][b] = sum_q w_q l_a'(eta_q) l_b'(eta_q),  M[a][b] = sum_q w_q l_a l_b
// Reflection: B[NQ-1-q][NP-1-a] = B[q][a], K and M centro-symmetric.
// Scaled tables (sc): every column (the input index a, and b of G1) divided
// by m_a = W_a (GLL weight), doubled on the two end nodes.  On a mesh of
// cells of one size the lumped mass of a DOF is det J prod_d m_{a_d} (an end
// node's weight comes from the two cells that share it), so contracting
// with the scaled tables along all three axes applies det J M_D^{-1} to the
// input first; m is symmetric, so the scaled tables keep the reflection
// symmetry.
//   BE[q][a] = (B[q][a] + B[q][NP-1-a]) / 2 (a < NP/2), B[q][mid] (a = mid)
//   BO[q][a] = (B[q][a] - B[q][NP-1-a]) / 2
// likewise KE/KO, ME/MO with the row index a in place of q.
template <int NP, int NQ>
struct Tables {
  static constexpr int PH = NP / 2, PC = (NP + 1) / 2, QH = NQ / 2, QC = (NQ + 1) / 2;
  double W[NP] = {};       // GLL weights (the lumped mass M_D of the element)
  double BE[QC][PC] = {};
  double BO[QH > 0 ? QH : 1][PH > 0 ? PH : 1] = {};
  double KE[PC][PC] = {};
  double KO[PH > 0 ? PH : 1][PH > 0 ? PH : 1] = {};
  double ME[PC][PC] = {};
  double MO[PH > 0 ? PH : 1][PH > 0 ? PH : 1] = {};
  double DG[NQ][NQ] = {};  // DG[i][j] = g_j'(eta_i), g_j the Lagrange basis through the Gauss points
  double G1[NP][NP] = {};  // G1[a][b] = sum_q w_q l_a(eta_q) l_b'(eta_q) (imaginary k term)
};

template <int NP, int NQ>
constexpr Tables<NP, NQ> make_tables(bool sc) {
  constexpr Rule<NP> xi = gll<NP - 1>();
  constexpr Rule<NQ> g = gauss<NQ>();
  double B[NQ][NP] = {}, D[NQ][NP] = {}, K[NP][NP] = {}, M[NP][NP] = {};
  for (int q = 0; q < NQ; ++q)
    for (int a = 0; a < NP; ++a) {
      double v = 1.0, d = 0.0;
      for (int j = 0; j < NP; ++j)
        if (j != a) v *= (g.x[q] - xi.x[j]) / (xi.x[a] - xi.x[j]);
      for (int m = 0; m < NP; ++m) {
        if (m == a) continue;
        double t = 1.0 / (xi.x[a] - xi.x[m]);
        for (int j = 0; j < NP; ++j)
          if (j != a && j != m) t *= (g.x[q] - xi.x[j]) / (xi.x[a] - xi.x[j]);
        d += t;
      }
      B[q][a] = v;
      D[q][a] = d;
    }
  Tables<NP, NQ> t{};
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) {
      double k = 0.0, m = 0.0, gi = 0.0;
      for (int q = 0; q < NQ; ++q) {
        k += g.w[q] * D[q][a] * D[q][b];
        m += g.w[q] * B[q][a] * B[q][b];
        gi += g.w[q] * B[q][a] * D[q][b];
      }
      K[a][b] = k;
      M[a][b] = m;
      t.G1[a][b] = gi;
    }
  for (int i = 0; i < NQ; ++i)
    for (int jj = 0; jj < NQ; ++jj) {
      double d = 0.0;
      for (int m = 0; m < NQ; ++m) {
        if (m == jj) continue;
        double tt = 1.0 / (g.x[jj] - g.x[m]);
        for (int k = 0; k < NQ; ++k)
          if (k != jj && k != m) tt *= (g.x[i] - g.x[k]) / (g.x[jj] - g.x[k]);
        d += tt;
      }
      t.DG[i][jj] = d;
    }
  for (int a = 0; a < NP; ++a) {
    const double P = legendre_P(NP - 1, xi.x[a]);
    t.W[a] = 2.0 / ((NP - 1) * NP * P * P);
  }
  if (sc) {
    for (int a = 0; a < NP; ++a) {
      const double inv = 1.0 / (t.W[a] * ((a == 0 || a == NP - 1) ? 2.0 : 1.0));
      for (int q = 0; q < NQ; ++q) B[q][a] *= inv;
      for (int r = 0; r < NP; ++r) {
        K[r][a] *= inv;
        M[r][a] *= inv;
        t.G1[r][a] *= inv;
      }
    }
  }
  constexpr int PH = NP / 2, PC = (NP + 1) / 2, QC = (NQ + 1) / 2, QH = NQ / 2;
  for (int q = 0; q < QC; ++q)
    for (int a = 0; a < PC; ++a) t.BE[q][a] = a < PH ? 0.5 * (B[q][a] + B[q][NP - 1 - a]) : B[q][a];
  for (int q = 0; q < QH; ++q)
    for (int a = 0; a < PH; ++a) t.BO[q][a] = 0.5 * (B[q][a] - B[q][NP - 1 - a]);
  for (int r = 0; r < PC; ++r)
    for (int a = 0; a < PC; ++a) {
      t.KE[r][a] = a < PH ? 0.5 * (K[r][a] + K[r][NP - 1 - a]) : K[r][a];
      t.ME[r][a] = a < PH ? 0.5 * (M[r][a] + M[r][NP - 1 - a]) : M[r][a];
    }
  for (int r = 0; r < PH; ++r)
    for (int a = 0; a < PH; ++a) {
      t.KO[r][a] = 0.5 * (K[r][a] - K[r][NP - 1 - a]);
      t.MO[r][a] = 0.5 * (M[r][a] - M[r][NP - 1 - a]);
    }
  return t;
}

template <int NP, int NQ>
struct Tab {
  static constexpr Tables<NP, NQ> t = make_tables<NP, NQ>(false);
  static constexpr Tables<NP, NQ> ts = make_tables<NP, NQ>(true);   // columns over m_a
};

}  // namespace ref1d

// compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1
template <typename F, int... I>
__host__ __device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  if constexpr (N > 0) sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---- 1-D contractions on one line (values in registers) ------------------------

template <typename T>
__host__ __device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return fmaf(a, b, c); else return fma(a, b, c);
}

// y[NQ] = B x[NP]  (SC: the scaled table)
template <int NP, int NQ, bool SC = false, typename T>
__host__ __device__ __forceinline__ void line_B(const T (&x)[NP], T (&y)[NQ]) {
  using TB = ref1d::Tab<NP, NQ>;
  constexpr int PH = NP / 2, PC = (NP + 1) / 2, QH = NQ / 2, QC = (NQ + 1) / 2;
  T e[PC], o[PH > 0 ? PH : 1];
  sfor<PH>([&](auto a) {
    e[a] = x[a] + x[NP - 1 - a];
    o[a] = x[a] - x[NP - 1 - a];
  });
  if constexpr (NP % 2) e[PC - 1] = x[PC - 1];
  sfor<QC>([&](auto q) {
    T ye = T(0);
    sfor<PC>([&](auto a) {
      constexpr T c = (T)(SC ? TB::ts.BE[q][a] : TB::t.BE[q][a]);
      ye = fma_t(c, e[a], ye);
    });
    if constexpr (q < QH) {
      T yo = T(0);
      sfor<PH>([&](auto a) {
        constexpr T c = (T)(SC ? TB::ts.BO[q][a] : TB::t.BO[q][a]);
        yo = fma_t(c, o[a], yo);
      });
      y[q] = ye + yo;
      y[NQ - 1 - q] = ye - yo;
    } else {
      y[q] = ye;
    }
  });
}

// x[NP] = B^T y[NQ]
template <int NP, int NQ, typename T>
__host__ __device__ __forceinline__ void line_Bt(const T (&y)[NQ], T (&x)[NP]) {
  using TB = ref1d::Tab<NP, NQ>;
  constexpr int PH = NP / 2, PC = (NP + 1) / 2, QH = NQ / 2, QC = (NQ + 1) / 2;
  T s[QC], d[QH > 0 ? QH : 1];
  sfor<QH>([&](auto q) {
    s[q] = y[q] + y[NQ - 1 - q];
    d[q] = y[q] - y[NQ - 1 - q];
  });
  if constexpr (NQ % 2) s[QC - 1] = y[QC - 1];
  sfor<PC>([&](auto a) {
    T xe = T(0);
    sfor<QC>([&](auto q) {
      constexpr T c = (T)TB::t.BE[q][a];
      xe = fma_t(c, s[q], xe);
    });
    if constexpr (a < PH) {
      T xo = T(0);
      sfor<QH>([&](auto q) {
        constexpr T c = (T)TB::t.BO[q][a];
        xo = fma_t(c, d[q], xo);
      });
      x[a] = xe + xo;
      x[NP - 1 - a] = xe - xo;
    } else {
      x[a] = xe;
    }
  });
}

// even / odd parts of a line of NP node values
template <int NP, typename T>
struct EOIn {
  T e[(NP + 1) / 2];
  T o[NP / 2 > 0 ? NP / 2 : 1];
};
template <int NP, typename T>
__host__ __device__ __forceinline__ EOIn<NP, T> split_eo(const T (&x)[NP]) {
  constexpr int PH = NP / 2, PC = (NP + 1) / 2;
  EOIn<NP, T> r;
  sfor<PH>([&](auto a) {
    r.e[a] = x[a] + x[NP - 1 - a];
    r.o[a] = x[a] - x[NP - 1 - a];
  });
  if constexpr (NP % 2) r.e[PC - 1] = x[PC - 1];
  return r;
}

// y = A x for a centro-symmetric NP x NP table (K1 if KT, else M1; SC: the
// scaled table), from the even / odd parts of x
template <int NP, int NQ, bool KT, bool SC = false, typename T>
__host__ __device__ __forceinline__ void line_sym(const EOIn<NP, T>& in, T (&y)[NP]) {
  using TB = ref1d::Tab<NP, NQ>;
  constexpr const ref1d::Tables<NP, NQ>& tb = SC ? TB::ts : TB::t;
  constexpr int PH = NP / 2, PC = (NP + 1) / 2;
  sfor<PC>([&](auto r) {
    T ye = T(0);
    sfor<PC>([&](auto a) {
      constexpr T c = (T)(KT ? tb.KE[r][a] : tb.ME[r][a]);
      ye = fma_t(c, in.e[a], ye);
    });
    if constexpr (r < PH) {
      T yo = T(0);
      sfor<PH>([&](auto a) {
        constexpr T c = (T)(KT ? tb.KO[r][a] : tb.MO[r][a]);
        yo = fma_t(c, in.o[a], yo);
      });
      y[r] = ye + yo;
      y[NP - 1 - r] = ye - yo;
    } else {
      y[r] = ye;
    }
  });
}

// y = G1 x on one line of NP node values (G1 is not symmetric: a plain
// product with compile-time coefficients; SC: the scaled table)
template <int NP, int NQ, bool SC = false, typename T>
__host__ __device__ __forceinline__ void line_g1(const T (&x)[NP], T (&y)[NP]) {
  using TB = ref1d::Tab<NP, NQ>;
  sfor<NP>([&](auto a) {
    T acc = T(0);
    sfor<NP>([&](auto b) {
      constexpr T c = (T)(SC ? TB::ts.G1[a][b] : TB::t.G1[a][b]);
      acc = fma_t(c, x[b], acc);
    });
    y[a] = acc;
  });
}

// t = v (Dg u) + Dg^T (v u) on one line of NQ quadrature values: the GGA
// term along one axis, with v = W_q det J (2/h) V_GGA along that axis.  The
// derivative of the FE field at the Gauss points is the collocation
// derivative through those points (exact: the field restricted to the line
// is a polynomial of degree NP - 1 < NQ).
template <int NP, int NQ, typename T>
__host__ __device__ __forceinline__ void line_gga(const T (&u)[NQ], const T (&v)[NQ], T (&t)[NQ]) {
  using TB = ref1d::Tab<NP, NQ>;
  T vu[NQ];
  sfor<NQ>([&](auto q) { vu[q] = v[q] * u[q]; });
  sfor<NQ>([&](auto i) {
    T du = T(0), dt = T(0);
    sfor<NQ>([&](auto j) {
      constexpr T c = (T)TB::t.DG[i][j];
      constexpr T ct = (T)TB::t.DG[j][i];
      du = fma_t(c, u[j], du);
      dt = fma_t(ct, vu[j], dt);
    });
    t[i] = fma_t(v[i], du, dt);
  });
}

// ---- LDS slabs ---------------------------------------------------------------------

// Columns per item: 8 in FP32, 4 in FP64 (so three workgroups fit in the LDS
// of a CU either way); the x index is padded to 9.
template <typename T>
constexpr int kCB = sizeof(T) == 4 ? 8 : 4;
// Threads per workgroup: 64 line slots of CB columns each, one line per
// thread and pass (FP32: 512 threads, so six waves per SIMD fit in the
// register file; FP64: 256)
template <typename T>
constexpr int kNT = 64 * kCB<T>;
// Kernel variants.
constexpr int kValuH = 0;        // K + V, every cell of one size (factors as arguments)
constexpr int kValuGenH = 1;     // K + V, per-cell geometry
constexpr int kValuGenHG = 2;    // K + V + the GGA term, per-cell geometry
constexpr int kValuGenMass = 3;  // det J_e M, times -lambda_n per column when lam is given
constexpr int kValuHRes = 4;     // K + V - lambda_n M, every cell of one size
// complex (k-point) operators, every cell of one size: the two modes above
// plus the imaginary k term s_n (Hi X)[n ^ 1] on the (re, im) column pairs
constexpr int kValuHC = 5;
constexpr int kValuHResC = 6;
constexpr int kValuMass = 7;     // det J M, every cell of one size (real and complex operators alike)
// Chebyshev step of the filter on cells of one size (real; complex with the
// imaginary k term): Y += alpha (K + V) M_D^{-1} X through the scaled 1-D
// tables, and at the first visit of each DOF the node part of the step
// applied to the old value of Y first (see the kernel)
constexpr int kValuStep = 8;
constexpr int kValuStepC = 9;
// the step on general operators (graded mesh; with the GGA term): per-cell
// geometry, and the gathered values at a cell's face nodes scaled by the
// ratio of the lumped mass the uniform tables assume to the DOF's own
// (the neighbour across a face may have another size)
constexpr int kValuGenStep = 10;
constexpr int kValuGenStepG = 11;
// variants that read the per-cell geometry table (and need it non-null)
constexpr bool is_general_mode(int mode) {
  return mode == kValuGenH || mode == kValuGenHG || mode == kValuGenMass || mode == kValuGenStep ||
         mode == kValuGenStepG;
}
static_assert(!is_general_mode(kValuH) && !is_general_mode(kValuHRes) && !is_general_mode(kValuHC) &&
                  !is_general_mode(kValuHResC) && !is_general_mode(kValuMass) && !is_general_mode(kValuStep) &&
                  !is_general_mode(kValuStepC),
              "uniform variants");
// Waves per SIMD the registers are held to: FP32 six (three workgroups of
// eight waves per CU, as many as the LDS holds), FP64 three; the GGA and the
// complex variants hold one or two more slabs in LDS (two workgroups per
// CU): FP32 four, FP64 two.  The FP32 step variant is held to four as
// well: the filter runs two blocks on two streams, and with six waves of
// the step kernel the other stream's kernels find no room (degree-6 filter
// pass of 1024 states: 0.585 s at four waves, 0.65 s at six).
template <typename T, int MODE>
constexpr int kWaves = (MODE == kValuGenHG || MODE == kValuHC || MODE == kValuHResC || MODE == kValuStepC ||
                        MODE == kValuGenStepG)
                           ? (sizeof(T) == 4 ? 4 : 2)
                       : (MODE == kValuStep || MODE == kValuGenStep) ? (sizeof(T) == 4 ? 4 : 3)
                                           : (sizeof(T) == 4 ? 6 : 3);
constexpr int kXP = 9;
// U: extents up to 8 x 8 x 8;  K, M: up to 7 x 7 x 7 (element offsets, col fastest)
template <typename T>
__host__ __device__ constexpr int offU(int x, int y, int z) { return ((z * 8 + y) * kXP + x) * kCB<T>; }
template <typename T>
__host__ __device__ constexpr int offK(int x, int y, int z) { return ((z * 7 + y) * kXP + x) * kCB<T>; }
template <typename T>
constexpr int kSlabU = 8 * 8 * kXP * kCB<T>;
template <typename T>
constexpr int kSlabK = 7 * 7 * kXP * kCB<T>;

// The R lines of one pass owned by a thread: line index L = slot + S r
// (S = 256 / CB slots) enumerates (u, v) = (L % NU, L / NU); lines past
// NU * NV are clamped to the last line: their loads stay in range, and the
// lanes skip their arithmetic and stores (whole waves skip when all of their
// lines are past the end).
template <int NU, int NV, int S, int R>
struct Lines {
  int u[R], v[R];
  bool on[R];
  __device__ __forceinline__ Lines(int slot) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int L = slot + S * r;
      on[r] = L < NU * NV;
      L = on[r] ? L : NU * NV - 1;
      u[r] = L % NU;
      v[r] = L / NU;
    }
  }
};

}  // namespace

template <typename T, int NP, int NQ, int MODE>
__global__ void __launch_bounds__(kNT<T>) __attribute__((amdgpu_waves_per_eu((kWaves<T, MODE>))))
k_cell_valu(CellArgs<T> A, int ncoltiles, int nitems, T fx, T fy, T fz) {
  constexpr bool GEN = is_general_mode(MODE);   // reads the per-cell table A.geo
  constexpr bool GGA = MODE == kValuGenHG || MODE == kValuGenStepG;
  constexpr bool MASS = MODE == kValuGenMass || MODE == kValuMass;
  constexpr bool RES = MODE == kValuHRes || MODE == kValuHResC;
  constexpr bool STEP = MODE == kValuStep || MODE == kValuStepC || MODE == kValuGenStep || MODE == kValuGenStepG;
  constexpr bool CPLX = MODE == kValuHC || MODE == kValuHResC || MODE == kValuStepC;
  constexpr bool SC = STEP;   // input-side 1-D contractions with the scaled tables
  static_assert(!(RES && GEN), "the residual mode uses the uniform factors");
  static_assert(!(CPLX && GEN), "complex operators use the uniform factors");
  static_assert(!(STEP && RES), "the step and residual modes are separate");
  constexpr int CB = kCB<T>;
  constexpr int NT = kNT<T>;
  constexpr int S = NT / CB;                   // line slots
  constexpr int R = (64 + S - 1) / S;          // lines per thread and pass (at most 64 lines)
  constexpr int NL = NP * NP * NP;
  constexpr int NQ3 = NQ * NQ * NQ;
  constexpr int NJ = (NL * CB + NT - 1) / NT;  // gathered elements per thread and item
  constexpr int NV = (NQ3 + NT - 1) / NT;      // V(q) W_q values per thread and item
  static_assert(NP <= 7 && NQ <= 8, "slab extents");
  __shared__ T sU[kSlabU<T>];
  __shared__ T sK[kSlabK<T>];
  __shared__ T sM[kSlabK<T>];
  __shared__ T vws[MASS ? 1 : NQ3];
  __shared__ T sG[GGA ? kSlabU<T> : 1];   // GGA: V u plus the GGA term at the quadrature points
  __shared__ T vgs[GGA ? 3 * NQ3 : 1];    // GGA: W det J (2/h_d) V_GGA,d of the item's cell
  __shared__ T sI[CPLX ? kSlabK<T> : 1];  // complex: the imaginary k term of the partner column
  const int tid = threadIdx.x;
  const int col = tid & (CB - 1);
  const int slot = tid / CB;

  // gathered local node l = slot + S j = (a, b, c): pk[j] = (row offset of
  // the node from the cell's first node << 15) | (byte offset in U); its
  // byte offset in K (the result) follows from the U offset (K has 7 y rows
  // per z where U has 8).  Threads past the last node carry a valid row and
  // store nothing.
  constexpr int kLdsBits = 15;
  static_assert(kSlabU<T> * (int)sizeof(T) <= (1 << kLdsBits), "U offsets must fit the field");
  const int p = NP - 1;
  const int Gx = A.n0 * p, Gy = A.n1 * p, Gz = A.n2 * p;
  const bool off_fits = (int64_t)p + (int64_t)Gx * (p + (int64_t)Gy * p) < (1 << (32 - kLdsBits));
  constexpr int kLast = (NL * CB) % NT == 0 ? NJ : NJ - 1;
  auto lnode = [&](int j) { return slot + S * j; };
  auto lreal = [&](int j) { return j < kLast || lnode(j) < NL; };
  unsigned pk[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = lreal(j) ? lnode(j) : 0;
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    pk[j] = ((off_fits ? (unsigned)(a + Gx * (b + Gy * c)) : 0u) << kLdsBits) |
            (unsigned)((offU<T>(a, b, c) + col) * (int)sizeof(T));
  }
  // step mode: the position class (0-26, 31 past the last node) of each of
  // the thread's gathered nodes, 5 bits per node in one register
  unsigned cls_pack = 0;
  if constexpr (STEP) {
    static_assert(NJ * 5 <= 32, "position classes must fit one register");
    auto cls1 = [](int a) { return a == 0 ? 0 : (a == NP - 1 ? 2 : 1); };
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int l = lnode(j);
      const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
      cls_pack |= (lreal(j) ? (unsigned)(cls1(a) + 3 * cls1(b) + 9 * cls1(c)) : 31u) << (5 * j);
    }
  }
  // byte offset in K of the element at byte offset u in U:
  // offU - offK = z * 9 * CB elements, z = u / (8 * 9 * CB * sizeof(T))
  auto k_of_u = [](unsigned u) -> int {
    constexpr unsigned zb = 8u * kXP * CB * sizeof(T);
    return (int)(u - (u / zb) * (kXP * CB * sizeof(T)));
  };
  static_assert(offU<T>(3, 5, 6) - offK<T>(3, 5, 6) == 6 * kXP * CB, "K offset from U offset");
  struct CellPos {
    int ci, cj, ck, e, base;
    bool inner;
  };
  auto cell_pos = [&](int packed) {
    CellPos cp;
    cp.ci = packed & 1023;
    cp.cj = (packed >> 10) & 1023;
    cp.ck = (packed >> 20) & 1023;
    cp.e = cp.ci + A.n0 * (cp.cj + A.n1 * cp.ck);
    cp.base = cp.ci * p + Gx * (cp.cj * p + Gy * cp.ck * p);
    cp.inner = off_fits && cp.ci + 1 < A.n0 && cp.cj + 1 < A.n1 && cp.ck + 1 < A.n2;
    return cp;
  };
  auto nodes_of = [&](const CellPos& cp, int (&node)[NJ]) {
    if (cp.inner) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) node[j] = cp.base + (int)(pk[j] >> kLdsBits);
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int l = lreal(j) ? lnode(j) : 0;
        const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
        int gx = cp.ci * p + a; gx = gx >= Gx ? gx - Gx : gx;
        int gy = cp.cj * p + b; gy = gy >= Gy ? gy - Gy : gy;
        int gz = cp.ck * p + c; gz = gz >= Gz ? gz - Gz : gz;
        node[j] = gx + Gx * (gy + Gy * gz);
      }
    }
  };
  const uint32_t ldxb = (uint32_t)(A.ldx * (int64_t)sizeof(T)), ldyb = (uint32_t)(A.ldy * (int64_t)sizeof(T));
  // element (row, column n) of a row-major block with a row stride of ldb bytes
  auto elem = [](auto* base, uint32_t ldb, int n, int row) {
    using P = decltype(base);
    using C = typename std::conditional<std::is_const<typename std::remove_pointer<P>::type>::value, const char,
                                        char>::type;
    return reinterpret_cast<P>(reinterpret_cast<C*>(base + n) + (uint64_t)(uint32_t)row * ldb);
  };

  // items (cell of the colour, column tile), cell-major; XCD x takes the
  // x-th eighth of them (block w runs on XCD w % 8); the cell list is read
  // through the scalar cache
  typedef const __attribute__((address_space(4))) int* ConstIntP;
  const ConstIntP cells = (ConstIntP)A.cells;
  const int xcd = blockIdx.x & 7;
  const int i_end = (int)((int64_t)nitems * (xcd + 1) / 8);
  const int i_step = gridDim.x >> 3;
  int item = (int)((int64_t)nitems * xcd / 8) + (blockIdx.x >> 3);
  const int st_c = i_step / ncoltiles, st_t = i_step % ncoltiles;
  int cur_c = item / ncoltiles, cur_t = item % ncoltiles;
  auto advance = [&](int& c, int& t) {
    c += st_c;
    t += st_t;
    if (t >= ncoltiles) {
      t -= ncoltiles;
      ++c;
    }
  };

  T xr[NJ], vr[MASS ? 1 : NV], gr[GGA ? 3 * NV : 1];
  auto load_item = [&](int c, int t) {
    const CellPos cp = cell_pos(cells[c]);
    const int n = t * CB + col;
    int node[NJ];
    nodes_of(cp, node);
    const int nn = n < A.ncols ? n : 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) xr[j] = *elem(A.X, ldxb, nn, node[j]);
    if constexpr (!MASS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int q = tid + NT * v;
        if (NQ3 % NT == 0 || q < NQ3) vr[v] = A.Vw[(int64_t)cp.e * NQ3 + q];
      }
    }
    if constexpr (GGA) {
#pragma unroll
      for (int v = 0; v < 3 * NV; ++v) {
        const int q = tid + NT * (v % NV);
        if (NQ3 % NT == 0 || q < NQ3) gr[v] = A.vg[((int64_t)cp.e * 3 + v / NV) * NQ3 + q];
      }
    }
  };
  // stage the gathered values of the item whose cell is cells[c]
  auto stage = [&](int c) {
    if constexpr (STEP && GEN) {
      // general step: a node on a face of the cell is scaled by the cell's
      // factor for that face (the uniform tables' lumped mass over the
      // DOF's own), per face the node lies on
      typedef const __attribute__((address_space(4))) T* ConstTP;
      const ConstTP r = (ConstTP)A.frho + 6 * cell_pos(cells[c]).e;
      T rf[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) rf[k] = r[k];
      unsigned cpk = cls_pack;   // opaque: the classes are unpacked here, not held per node
      asm volatile("" : "+v"(cpk));
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const unsigned cl = (cpk >> (5 * j)) & 31u;
        const unsigned ca = cl % 3u, cb = (cl / 3u) % 3u, cc = cl / 9u;
        const T fa = ca == 0 ? rf[0] : (ca == 2 ? rf[1] : T(1));
        const T fb = cb == 0 ? rf[2] : (cb == 2 ? rf[3] : T(1));
        const T fc = cc == 0 ? rf[4] : (cc == 2 ? rf[5] : T(1));
        if (lreal(j))
          *reinterpret_cast<T*>(reinterpret_cast<char*>(sU) + (pk[j] & ((1u << kLdsBits) - 1))) = xr[j] * (fa * fb * fc);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (lreal(j)) *reinterpret_cast<T*>(reinterpret_cast<char*>(sU) + (pk[j] & ((1u << kLdsBits) - 1))) = xr[j];
      }
    }
    if constexpr (!MASS) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (NQ3 % NT == 0 || tid + NT * v < NQ3) vws[tid + NT * v] = vr[v];
    }
    if constexpr (GGA) {
#pragma unroll
      for (int v = 0; v < 3 * NV; ++v)
        if (NQ3 % NT == 0 || tid + NT * (v % NV) < NQ3) vgs[(v / NV) * NQ3 + tid + NT * (v % NV)] = gr[v];
    }
  };

  if (item < i_end) load_item(cur_c, cur_t);
  __syncthreads();
  if (item < i_end) stage(cur_c);
  __syncthreads();

  for (; item < i_end; item += i_step) {
    const int n = cur_t * CB + col;
    const bool valid = n < A.ncols;
    const CellPos cp = cell_pos(cells[cur_c]);
    // the line of each pass is recomputed from the slot in every item (a few
    // integer operations) rather than held in registers across the loop
    int lslot = slot;
    asm volatile("" : "+v"(lslot));
    // FP32 step mode: the old output rows are read at the assembly (the
    // registers that would hold them across the passes are what the step's
    // own loads need there)
    constexpr bool kLateYo = STEP && sizeof(T) == 4;
    T yo[NJ];
    if constexpr (!kLateYo) {
      int node[NJ];
      nodes_of(cp, node);
      const int nn = valid ? n : 0;
#pragma unroll
      for (int j = 0; j < NJ; ++j) yo[j] = *elem(A.Y, ldyb, nn, node[j]);
    }
    // step mode: which of the thread's nodes this cell visits first (the
    // cell of the lowest colour sharing a DOF), this item's gathered X (kept
    // from the registers the next item's prefetch overwrites) and the FP64
    // residual block at those nodes
    unsigned sown = 0;
    T sxv[STEP ? NJ : 1];
    double syf[STEP ? NJ : 1];
    if constexpr (STEP) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) sxv[j] = xr[j];
    }
    auto step_loads = [&](const int (&node)[NJ]) {
      typedef const __attribute__((address_space(4))) unsigned* ConstUP;
      const unsigned cm = ((ConstUP)A.own)[cp.e];
      // the classes are unpacked here in every item (one register held
      // across the loop instead of one per node)
      unsigned cpk = cls_pack;
      asm volatile("" : "+v"(cpk));
#pragma unroll
      for (int j = 0; j < NJ; ++j) sown |= ((cm >> ((cpk >> (5 * j)) & 31u)) & 1u) << j;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        syf[j] = 0.0;
        if ((sown >> j) & 1u) syf[j] = A.y64[(int64_t)node[j] * A.ldy64 + n];
      }
    };
    // FP32 step mode: the first-visit FP64 rows are requested here and wait
    // in registers through the passes (FP64: at the assembly; requested
    // here they cost more than they hide, pass of 1024 states 1.08 against
    // 0.975 s, where FP32 gains 0.556 -> 0.548 s)
    constexpr bool kEarlyY = STEP && sizeof(T) == 4;
    if constexpr (kEarlyY) {
      if (valid) {
        int node[NJ];
        nodes_of(cp, node);
        step_loads(node);
      }
    }
    int nxt_c = cur_c, nxt_t = cur_t;
    advance(nxt_c, nxt_t);
    const bool more = item + i_step < i_end;
    load_item(more ? nxt_c : cur_c, more ? nxt_t : cur_t);
    // kinetic factors 1/2 det J (2/h_d)^2 and det J: the cell's own on a
    // general operator (read through the scalar cache), else the arguments
    T ifx = fx, ify = fy, ifz = fz, idet = A.detJ;
    if constexpr (GEN) {
      typedef const __attribute__((address_space(4))) T* ConstTP;
      const ConstTP g = (ConstTP)A.geo + 4 * cp.e;
      ifx = g[0];
      ify = g[1];
      ifz = g[2];
      idet = g[3];
    }

    // P1 x: lines (b, c); U -> B U (in place), K1 U -> K, M1 U -> M
    // (mass: M1 U -> M only; complex: also I <- G1 U' of the partner column)
    {
      const Lines<NP, NP, S, R> ln(lslot);
      T x[R][NP], xp[CPLX ? R : 1][NP];
#pragma unroll
      for (int r = 0; r < R; ++r) sfor<NP>([&](auto a) { x[r][a] = sU[offU<T>(a, ln.u[r], ln.v[r]) + col]; });
      if constexpr (CPLX) {
        // the partner column's line (the neighbouring lane of this wave
        // overwrites it below: its load is issued before any store)
#pragma unroll
        for (int r = 0; r < R; ++r) sfor<NP>([&](auto a) { xp[r][a] = sU[offU<T>(a, ln.u[r], ln.v[r]) + (col ^ 1)]; });
        asm volatile("" ::: "memory");
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!ln.on[r]) continue;
        if constexpr (CPLX) {
          T yi[NP];
          line_g1<NP, NQ, SC>(xp[r], yi);
          sfor<NP>([&](auto a) { sI[offK<T>(a, ln.u[r], ln.v[r]) + col] = yi[a]; });
        }
        // each result is stored as soon as it is formed (fewer live registers)
        const EOIn<NP, T> eo = split_eo<NP>(x[r]);
        if constexpr (!MASS) {
          T yk[NP];
          line_sym<NP, NQ, true, SC>(eo, yk);
          sfor<NP>([&](auto a) { sK[offK<T>(a, ln.u[r], ln.v[r]) + col] = yk[a]; });
        }
        {
          T ym[NP];
          line_sym<NP, NQ, false, SC>(eo, ym);
          sfor<NP>([&](auto a) { sM[offK<T>(a, ln.u[r], ln.v[r]) + col] = ym[a]; });
        }
        if constexpr (!MASS) {
          T yb[NQ];
          line_B<NP, NQ, SC>(x[r], yb);
          sfor<NQ>([&](auto q) { sU[offU<T>(q, ln.u[r], ln.v[r]) + col] = yb[q]; });
        }
      }
    }
    __syncthreads();
    if constexpr (!MASS) {
      // P2 y: lines (qx, c): By
      {
        const Lines<NQ, NP, S, R> ln(lslot);
        T x[R][NP];
#pragma unroll
        for (int r = 0; r < R; ++r) sfor<NP>([&](auto b) { x[r][b] = sU[offU<T>(ln.u[r], b, ln.v[r]) + col]; });
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!ln.on[r]) continue;
          T y[NQ];
          line_B<NP, NQ, SC>(x[r], y);
          sfor<NQ>([&](auto q) { sU[offU<T>(ln.u[r], q, ln.v[r]) + col] = y[q]; });
        }
      }
      __syncthreads();
      if constexpr (!GGA) {
        // P3 + P4 z: lines (qx, qy): Bz, times V(q) W_q, then Bz^T, in
        // registers (both passes run on the same lines, so the line stays
        // with its thread and needs no barrier in between)
        const Lines<NQ, NQ, S, R> ln(lslot);
        T x[R][NP];
#pragma unroll
        for (int r = 0; r < R; ++r) sfor<NP>([&](auto c) { x[r][c] = sU[offU<T>(ln.u[r], ln.v[r], c) + col]; });
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!ln.on[r]) continue;
          T y[NQ];
          line_B<NP, NQ, SC>(x[r], y);
          const int q0 = ln.u[r] + NQ * ln.v[r];
          sfor<NQ>([&](auto q) { y[q] = y[q] * vws[q0 + NQ * NQ * q]; });
          T xo[NP];
          line_Bt<NP, NQ>(y, xo);
          sfor<NP>([&](auto c) { sU[offU<T>(ln.u[r], ln.v[r], c) + col] = xo[c]; });
        }
        __syncthreads();
      } else {
        // P3 z: lines (qx, qy): Bz (the field u at the quadrature points); u
        // stays in U and V(q) W_q u plus the z part of the GGA term go to G
        {
          const Lines<NQ, NQ, S, R> ln(lslot);
          T x[R][NP];
#pragma unroll
          for (int r = 0; r < R; ++r) sfor<NP>([&](auto c) { x[r][c] = sU[offU<T>(ln.u[r], ln.v[r], c) + col]; });
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (!ln.on[r]) continue;
            T y[NQ];
            line_B<NP, NQ, SC>(x[r], y);
            const int q0 = ln.u[r] + NQ * ln.v[r];
            T v[NQ], t[NQ];
            sfor<NQ>([&](auto q) { v[q] = vgs[2 * NQ3 + q0 + NQ * NQ * q]; });
            line_gga<NP, NQ>(y, v, t);
            sfor<NQ>([&](auto q) {
              sU[offU<T>(ln.u[r], ln.v[r], q) + col] = y[q];
              sG[offU<T>(ln.u[r], ln.v[r], q) + col] = fma_t(y[q], vws[q0 + NQ * NQ * q], t[q]);
            });
          }
        }
        __syncthreads();
        {
          // G += the y part of the GGA term: lines (qx, qz) along y
          {
            const Lines<NQ, NQ, S, R> ln(lslot);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if (!ln.on[r]) continue;
              T u[NQ], v[NQ], t[NQ];
              sfor<NQ>([&](auto q) {
                u[q] = sU[offU<T>(ln.u[r], q, ln.v[r]) + col];
                v[q] = vgs[NQ3 + ln.u[r] + NQ * (q + NQ * ln.v[r])];
              });
              line_gga<NP, NQ>(u, v, t);
              sfor<NQ>([&](auto q) { sG[offU<T>(ln.u[r], q, ln.v[r]) + col] += t[q]; });
            }
          }
          __syncthreads();
          // G += the x part: lines (qy, qz) along x
          {
            const Lines<NQ, NQ, S, R> ln(lslot);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if (!ln.on[r]) continue;
              T u[NQ], v[NQ], t[NQ];
              sfor<NQ>([&](auto q) {
                u[q] = sU[offU<T>(q, ln.u[r], ln.v[r]) + col];
                v[q] = vgs[q + NQ * (ln.u[r] + NQ * ln.v[r])];
              });
              line_gga<NP, NQ>(u, v, t);
              sfor<NQ>([&](auto q) { sG[offU<T>(q, ln.u[r], ln.v[r]) + col] += t[q]; });
            }
          }
          __syncthreads();
        }
        // P4 z: lines (qx, qy): Bz^T of G
        {
          const T* src = sG;
          const Lines<NQ, NQ, S, R> ln(lslot);
          T y[R][NQ];
#pragma unroll
          for (int r = 0; r < R; ++r) sfor<NQ>([&](auto q) { y[r][q] = src[offU<T>(ln.u[r], ln.v[r], q) + col]; });
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (!ln.on[r]) continue;
            T x[NP];
            line_Bt<NP, NQ>(y[r], x);
            sfor<NP>([&](auto c) { sU[offU<T>(ln.u[r], ln.v[r], c) + col] = x[c]; });
          }
        }
        __syncthreads();
      }
      // P5 y: lines (qx, c): By^T
      {
        const Lines<NQ, NP, S, R> ln(lslot);
        T y[R][NQ];
#pragma unroll
        for (int r = 0; r < R; ++r) sfor<NQ>([&](auto q) { y[r][q] = sU[offU<T>(ln.u[r], q, ln.v[r]) + col]; });
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!ln.on[r]) continue;
          T x[NP];
          line_Bt<NP, NQ>(y[r], x);
          sfor<NP>([&](auto b) { sU[offU<T>(ln.u[r], b, ln.v[r]) + col] = x[b]; });
        }
      }
      __syncthreads();
      // P6 x: lines (b, c): Bx^T -> U (the V term)
      {
        const Lines<NP, NP, S, R> ln(lslot);
        T y[R][NQ];
#pragma unroll
        for (int r = 0; r < R; ++r) sfor<NQ>([&](auto q) { y[r][q] = sU[offU<T>(q, ln.u[r], ln.v[r]) + col]; });
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!ln.on[r]) continue;
          T x[NP];
          line_Bt<NP, NQ>(y[r], x);
          sfor<NP>([&](auto a) { sU[offU<T>(a, ln.u[r], ln.v[r]) + col] = x[a]; });
        }
      }
    }
    // P7 y (kinetic; K and M are not touched by P2-P6, so no barrier is
    // needed before it): lines (a, c); K <- fx M1 K + fy K1 M,  M <- M1 M;
    // complex: I <- gx M1 I + gy G1 M' (M' the partner column's M)
    {
      const Lines<NP, NP, S, R> ln(lslot);
      T k[R][NP], m[R][NP], mp[CPLX ? R : 1][NP], iv[CPLX ? R : 1][NP];
#pragma unroll
      for (int r = 0; r < R; ++r)
        sfor<NP>([&](auto b) {
          if constexpr (!MASS) k[r][b] = sK[offK<T>(ln.u[r], b, ln.v[r]) + col];
          m[r][b] = sM[offK<T>(ln.u[r], b, ln.v[r]) + col];
        });
      if constexpr (CPLX) {   // the partner's M line is overwritten below by its lane
#pragma unroll
        for (int r = 0; r < R; ++r)
          sfor<NP>([&](auto b) {
            mp[r][b] = sM[offK<T>(ln.u[r], b, ln.v[r]) + (col ^ 1)];
            iv[r][b] = sI[offK<T>(ln.u[r], b, ln.v[r]) + col];
          });
        asm volatile("" ::: "memory");
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!ln.on[r]) continue;
        if constexpr (CPLX) {
          T mi[NP], gm[NP];
          line_sym<NP, NQ, false, SC>(split_eo<NP>(iv[r]), mi);
          line_g1<NP, NQ, SC>(mp[r], gm);
          sfor<NP>([&](auto b) { sI[offK<T>(ln.u[r], b, ln.v[r]) + col] = fma_t(A.gk[0], mi[b], A.gk[1] * gm[b]); });
        }
        const EOIn<NP, T> em = split_eo<NP>(m[r]);
        if constexpr (!MASS) {
          T mk[NP], km[NP];
          line_sym<NP, NQ, false, SC>(split_eo<NP>(k[r]), mk);
          line_sym<NP, NQ, true, SC>(em, km);
          sfor<NP>([&](auto b) { sK[offK<T>(ln.u[r], b, ln.v[r]) + col] = fma_t(ifx, mk[b], ify * km[b]); });
        }
        T mm[NP];
        line_sym<NP, NQ, false, SC>(em, mm);
        sfor<NP>([&](auto b) { sM[offK<T>(ln.u[r], b, ln.v[r]) + col] = mm[b]; });
      }
    }
    __syncthreads();
    // P8 z: lines (a, b): K <- U + M1 K + fz K1 M (the cell result);
    // mass: K <- M1 M; complex: plus s_n (M1 I + gz G1 M'), s_n = -1 on real
    // and +1 on imaginary columns
    {
      const Lines<NP, NP, S, R> ln(lslot);
      T k[R][NP], m[R][NP], mp[CPLX ? R : 1][NP], iv[CPLX ? R : 1][NP];
#pragma unroll
      for (int r = 0; r < R; ++r)
        sfor<NP>([&](auto c) {
          if constexpr (!MASS) k[r][c] = sK[offK<T>(ln.u[r], ln.v[r], c) + col];
          m[r][c] = sM[offK<T>(ln.u[r], ln.v[r], c) + col];
          if constexpr (CPLX) {
            mp[r][c] = sM[offK<T>(ln.u[r], ln.v[r], c) + (col ^ 1)];
            iv[r][c] = sI[offK<T>(ln.u[r], ln.v[r], c) + col];
          }
        });
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!ln.on[r]) continue;
        T acc[NP];
        if constexpr (MASS) {
          line_sym<NP, NQ, false, SC>(split_eo<NP>(m[r]), acc);
          sfor<NP>([&](auto c) { sK[offK<T>(ln.u[r], ln.v[r], c) + col] = acc[c]; });
        } else {
          line_sym<NP, NQ, false, SC>(split_eo<NP>(k[r]), acc);
          const EOIn<NP, T> em = split_eo<NP>(m[r]);
          {
            T km[NP];
            line_sym<NP, NQ, true, SC>(em, km);
            sfor<NP>([&](auto c) { acc[c] = fma_t(ifz, km[c], acc[c]); });
          }
          if constexpr (RES) {   // - lambda_n det J M1 M (the S part of the residual, local term)
            T mm[NP];
            line_sym<NP, NQ, false, SC>(em, mm);
            const T ml = valid ? -(T)A.lam[n] * idet : T(0);
            sfor<NP>([&](auto c) { acc[c] = fma_t(ml, mm[c], acc[c]); });
          }
          if constexpr (CPLX) {
            T mi[NP], gm[NP];
            line_sym<NP, NQ, false, SC>(split_eo<NP>(iv[r]), mi);
            line_g1<NP, NQ, SC>(mp[r], gm);
            const T sg = (col & 1) ? T(1) : T(-1);
            sfor<NP>([&](auto c) { acc[c] = fma_t(sg, fma_t(A.gk[2], gm[c], mi[c]), acc[c]); });
          }
          sfor<NP>([&](auto c) {
            sK[offK<T>(ln.u[r], ln.v[r], c) + col] = acc[c] + sU[offU<T>(ln.u[r], ln.v[r], c) + col];
          });
        }
      }
    }
    __syncthreads();
    // the next item's values into U (free now), then this item's assembly:
    // colour-ordered read-modify-write of CB contiguous columns per DOF
    stage(more ? nxt_c : cur_c);
    if (valid) {
      T f = A.alpha;
      if constexpr (STEP && GEN) f = f / idet;   // the cell's det J of M_D^{-1}
      if constexpr (MASS) f = f * idet * (A.lam ? (T)(-A.lam[n]) : T(1));
      int node[NJ];
      nodes_of(cp, node);
      if constexpr (STEP) {
        // Node part of the Chebyshev step at the first visit of a DOF, on
        // the old value before any cell adds to it:
        //   Y <- (-ac X - zz Y) + a lamY_n Yres
        // the last product and sum in FP64, rounded once
        if constexpr (kLateYo) {
#pragma unroll
          for (int j = 0; j < NJ; ++j) yo[j] = lreal(j) ? *elem(A.Y, ldyb, n, node[j]) : T(0);
        }
        if constexpr (!kEarlyY) step_loads(node);
        const double ly = A.sa * A.lamY[n];
        const T mac = (T)(-A.sac), zz = (T)A.szz;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {   // branch-free: a select per node
          const T part = mac * sxv[j] - zz * yo[j];
          const T upd = (T)((double)part + syf[j] * ly);
          yo[j] = ((sown >> j) & 1u) ? upd : yo[j];
        }
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (lreal(j))
          *elem(A.Y, ldyb, n, node[j]) =
              yo[j] + f * *reinterpret_cast<const T*>(reinterpret_cast<const char*>(sK) +
                                                      k_of_u(pk[j] & ((1u << kLdsBits) - 1)));
    }
    __syncthreads();
    cur_c = nxt_c;
    cur_t = nxt_t;
  }
}

namespace {

template <auto K, int NT>
int valu_grid(int nitems) {
  static const int resident = [] {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
      ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K, NT, 0) != hipSuccess || per_cu <= 0) per_cu = 1;
    return std::max(8, ncu * per_cu / 8 * 8);
  }();
  return std::max(8, std::min(resident, (nitems + 7) / 8 * 8));
}

template <typename T, int NP, int NQ, int MODE>
pawfe_status run_cell_valu(const pawfe_op* op, const CellArgs<T>& a0, hipStream_t s) {
  constexpr int CB = kCB<T>;
  CellArgs<T> a = a0;
  a.detJ = (T)op->detJ;
  for (int d = 0; d < 3; ++d) a.gk[d] = (T)(-op->kpt[d] * op->detJ * (2.0 / op->h[d]));
  if ((MODE == kValuHC || MODE == kValuHResC) && !op->cplx)
    return fail(PAWFE_EINVAL, "internal: complex cell variant on a real operator");
  if (is_general_mode(MODE) && !a.geo) return fail(PAWFE_EINVAL, "internal: general cell variant without geometry");
  if ((MODE == kValuGenHG || MODE == kValuGenStepG) && !a.vg)
    return fail(PAWFE_EINVAL, "internal: GGA cell variant without its table");
  if ((MODE == kValuGenStep || MODE == kValuGenStepG) && !a.frho)
    return fail(PAWFE_EINVAL, "internal: general step variant without its face factors");
  if ((MODE == kValuHRes || MODE == kValuHResC) && !a.lam)
    return fail(PAWFE_EINVAL, "internal: residual cell variant without lambda");
  if ((MODE == kValuStep || MODE == kValuStepC || MODE == kValuGenStep || MODE == kValuGenStepG) &&
      (!a.own || !a.y64 || !a.lamY))
    return fail(PAWFE_EINVAL, "internal: step cell variant without its tables");
  if (MODE == kValuStepC && !op->cplx) return fail(PAWFE_EINVAL, "internal: complex step variant on a real operator");
  const int ncoltiles = (a.ncols + CB - 1) / CB;
  const T fx = (T)(0.5 * op->detJ * (2.0 / op->h[0]) * (2.0 / op->h[0]));
  const T fy = (T)(0.5 * op->detJ * (2.0 / op->h[1]) * (2.0 / op->h[1]));
  const T fz = (T)(0.5 * op->detJ * (2.0 / op->h[2]) * (2.0 / op->h[2]));
  for (int c = 0; c < op->ncolour; ++c) {
    const int c0 = op->colour_off[c], c1 = op->colour_off[c + 1];
    if (c1 == c0) continue;
    CellArgs<T> ac = a;
    ac.cells = op->d.cell_pack + c0;
    const int nitems = (c1 - c0) * ncoltiles;
    const dim3 grid(valu_grid<k_cell_valu<T, NP, NQ, MODE>, kNT<T>>(nitems)), block(kNT<T>);
    hipLaunchKernelGGL((k_cell_valu<T, NP, NQ, MODE>), grid, block, 0, s, ac, ncoltiles, nitems, fx, fy, fz);
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

template <typename T, int MODE>
pawfe_status run_by_degree(const pawfe_op* op, const CellArgs<T>& a, hipStream_t s) {
  switch (op->p) {
    case 2: return run_cell_valu<T, 3, 4, MODE>(op, a, s);
    case 3: return run_cell_valu<T, 4, 5, MODE>(op, a, s);
    case 4: return run_cell_valu<T, 5, 6, MODE>(op, a, s);
    case 5: return run_cell_valu<T, 6, 7, MODE>(op, a, s);
    case 6: return run_cell_valu<T, 7, 8, MODE>(op, a, s);
    default: return fail(PAWFE_EUNSUPPORTED, "degree not compiled");
  }
}

// Local terms of a general operator (graded mesh and / or the GGA term), all
// on the vector ALUs: kModeH -> K + V [+ GGA]; kModeMass -> M (a.lam unused);
// kModeHRes -> K + V [+ GGA], then -lambda_n M per column.
template <typename T>
pawfe_status launch_cell_gen_impl(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s) {
  if (a.ldx < 0 || a.ldy < 0 || a.ldx * (int64_t)sizeof(T) >= (int64_t(1) << 32) ||
      a.ldy * (int64_t)sizeof(T) >= (int64_t(1) << 32))
    return fail(PAWFE_EINVAL, "row stride of 4 GiB or more");
  if (op->nq != op->p + 2) return fail(PAWFE_EUNSUPPORTED, "general operators need nq = p + 2");
  if (mode == kModeImg) return fail(PAWFE_EUNSUPPORTED, "complex general operators are not built");
  CellArgs<T> c = a;
  c.geo = std::is_same<T, double>::value ? (const T*)op->d.geo : (const T*)op->d.geo_f;
  c.vg = std::is_same<T, double>::value ? (const T*)op->d.vg : (const T*)op->d.vg_f;
  if (mode == kModeH || mode == kModeHRes) {
    CellArgs<T> h = c;
    h.lam = nullptr;
    const pawfe_status st = op->gga ? run_by_degree<T, kValuGenHG>(op, h, s) : run_by_degree<T, kValuGenH>(op, h, s);
    if (st != PAWFE_OK) return st;
  }
  if (mode == kModeMass || mode == kModeHRes) {
    CellArgs<T> m = c;
    m.lam = mode == kModeHRes ? a.lam : nullptr;
    return run_by_degree<T, kValuGenMass>(op, m, s);
  }
  return PAWFE_OK;
}

}  // namespace

}  // namespace pawfe
