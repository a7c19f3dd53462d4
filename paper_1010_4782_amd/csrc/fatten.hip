// Link fattening in FP64: the one-hop (fat) links of the asqtad action and the three-hop (long)
// products, from a thin gauge field in the user layout [4][Lt][Lz][Ly][Lx][3][3] complex128.
//
// The improved staggered operator of the paper (Sec. 1 and Sec. 2, the MILC setting) takes smeared
// one-hop links and three-hop Naik links as input.  The smearing recipe is the published asqtad one
// (Orginos, Toussaint and Sugar 1999; Lepage 1999): for direction mu,
//   V_mu = c1 U_mu + c3 (3-link staples) + c5 (5-link staples) + c7 (7-link staples) + cL (Lepage paths)
// with c1 = 5/8, c3 = 1/16, c5 = 1/64, c7 = 1/384, cL = -1/16, each path of l links scaled by u0^(1-l),
// and W_mu(n) = U_mu(n) U_mu(n+mu) U_mu(n+2mu).
//
// The staples are built in stages, as products of whole fields, instead of walking 85 paths per site:
// a "wrap" of a field F (a path from n to n+mu) in a transverse direction nu and sign s is
//   s = +1:  U_nu(n) F(n+nu) U_nu(n+mu)^dag,        s = -1:  U_nu(n-nu)^dag F(n-nu) U_nu(n-nu+mu),
// the path that steps s nu, follows F, and steps back.  With X_nu = wrap_nu^+(U_mu) + wrap_nu^-(U_mu)
// (the 3-link staples of one transverse direction):
//   3-link  = sum_nu X_nu
//   5-link  = sum_{rho != si} (wrap_rho^+ + wrap_rho^-)(X_si)
//   7-link  = sum_{rho != si, nu the third} (wrap_nu^+ + wrap_nu^-)((wrap_rho^+ + wrap_rho^-)(X_si))
//   Lepage  = sum_nu [wrap_nu^+(wrap_nu^+(U_mu)) + wrap_nu^-(wrap_nu^-(U_mu))]
// since a wrap is linear in F and the sum over the signs of each step factorises.  Per direction mu that
// is 28 passes over the lattice (each a few 3x3 products per site), instead of ~400 products per site.
// Every pass is one thread per site with the matrices in registers; all of them are HBM streams of
// 144-byte matrices (AoS, as the user layout stores them).
#include <hip/hip_runtime.h>

#include "fatten.h"

namespace stag {

namespace {

struct M3 {
  double2 e[9];  // row-major, (re, im)
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
// conj(a) * b
__device__ __forceinline__ double2 ccmul(double2 a, double2 b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }

__device__ __forceinline__ M3 ld(const double2* p) {
  M3 m;
#pragma unroll
  for (int i = 0; i < 9; ++i) m.e[i] = p[i];
  return m;
}
__device__ __forceinline__ void st(double2* p, const M3& m) {
#pragma unroll
  for (int i = 0; i < 9; ++i) p[i] = m.e[i];
}

// A B
__device__ __forceinline__ M3 mul_nn(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = cmul(a.e[3 * i], b.e[j]);
#pragma unroll
      for (int k = 1; k < 3; ++k) {
        const double2 t = cmul(a.e[3 * i + k], b.e[3 * k + j]);
        s.x += t.x;
        s.y += t.y;
      }
      c.e[3 * i + j] = s;
    }
  return c;
}
// A B^dag: (A B^dag)_ij = sum_k A_ik conj(B_jk)
__device__ __forceinline__ M3 mul_na(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = cmulc(a.e[3 * i], b.e[3 * j]);
#pragma unroll
      for (int k = 1; k < 3; ++k) {
        const double2 t = cmulc(a.e[3 * i + k], b.e[3 * j + k]);
        s.x += t.x;
        s.y += t.y;
      }
      c.e[3 * i + j] = s;
    }
  return c;
}
// A^dag B: (A^dag B)_ij = sum_k conj(A_ki) B_kj
__device__ __forceinline__ M3 mul_an(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = ccmul(a.e[i], b.e[j]);
#pragma unroll
      for (int k = 1; k < 3; ++k) {
        const double2 t = ccmul(a.e[3 * k + i], b.e[3 * k + j]);
        s.x += t.x;
        s.y += t.y;
      }
      c.e[3 * i + j] = s;
    }
  return c;
}

struct FGeo {
  int L[4];
  long stride[4];  // lex distance of one step: 1, Lx, Lx Ly, Lx Ly Lz
  long vol;
};

// lex index of n + d e_dir (periodic); c = coordinates of n
__device__ __forceinline__ long step(long lex, const int c[4], const FGeo& g, int dir, int d) {
  int v = c[dir] + d;
  v = v >= g.L[dir] ? v - g.L[dir] : (v < 0 ? v + g.L[dir] : v);
  return lex + (long)(v - c[dir]) * g.stride[dir];
}

__device__ __forceinline__ void coords(long lex, const FGeo& g, int c[4]) {
  c[0] = (int)(lex % g.L[0]);
  long r = lex / g.L[0];
  c[1] = (int)(r % g.L[1]);
  r /= g.L[1];
  c[2] = (int)(r % g.L[2]);
  c[3] = (int)(r / g.L[2]);
}

__device__ __forceinline__ const double2* mat(const double2* f, long site) { return f + 9 * site; }
__device__ __forceinline__ double2* mat(double2* f, long site) { return f + 9 * site; }

// out(n) = [acc ? out(n) : 0] + cw * sum over the signs in `signs` (bit 0: +, bit 1: -) of wrap_nu^s(F)(n);
// and, if out2 is not null, out2(n) += c2 * (the same sum).
__global__ __launch_bounds__(256) void k_wrap(const double2* __restrict__ U, const double2* __restrict__ F,
                                              double2* __restrict__ out, double cw, int acc,
                                              double2* __restrict__ out2, double c2, int mu, int nu, int signs,
                                              FGeo g) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.vol) return;
  int c[4];
  coords(n, g, c);
  const double2* Unu = U + 9 * (long)nu * g.vol;
  M3 s;
#pragma unroll
  for (int i = 0; i < 9; ++i) s.e[i] = {0.0, 0.0};
  if (signs & 1) {
    const long a = step(n, c, g, nu, 1);   // n + nu
    const long b = step(n, c, g, mu, 1);   // n + mu
    const M3 t = mul_nn(ld(mat(Unu, n)), ld(mat(F, a)));
    const M3 w = mul_na(t, ld(mat(Unu, b)));
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      s.e[i].x += w.e[i].x;
      s.e[i].y += w.e[i].y;
    }
  }
  if (signs & 2) {
    const long a = step(n, c, g, nu, -1);  // n - nu
    int ca[4] = {c[0], c[1], c[2], c[3]};
    ca[nu] = ca[nu] == 0 ? g.L[nu] - 1 : ca[nu] - 1;
    const long b = step(a, ca, g, mu, 1);  // n - nu + mu
    const M3 t = mul_an(ld(mat(Unu, a)), ld(mat(F, a)));
    const M3 w = mul_nn(t, ld(mat(Unu, b)));
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      s.e[i].x += w.e[i].x;
      s.e[i].y += w.e[i].y;
    }
  }
  double2* o = mat(out, n);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double2 prev = acc ? o[i] : double2{0.0, 0.0};
    o[i] = {prev.x + cw * s.e[i].x, prev.y + cw * s.e[i].y};
  }
  if (out2) {
    double2* o2 = mat(out2, n);
#pragma unroll
    for (int i = 0; i < 9; ++i) o2[i] = {o2[i].x + c2 * s.e[i].x, o2[i].y + c2 * s.e[i].y};
  }
}

// X = P + M;  V += c3 X
__global__ __launch_bounds__(256) void k_staple_sum(const double2* __restrict__ P, const double2* __restrict__ M,
                                                    double2* __restrict__ X, double2* __restrict__ V, double c3,
                                                    long n9) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n9) return;
  const double2 x = {P[i].x + M[i].x, P[i].y + M[i].y};
  X[i] = x;
  V[i] = {V[i].x + c3 * x.x, V[i].y + c3 * x.y};
}

// V = c1 U
__global__ __launch_bounds__(256) void k_scale(const double2* __restrict__ U, double2* __restrict__ V, double c1,
                                               long n9) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n9) return;
  V[i] = {c1 * U[i].x, c1 * U[i].y};
}

// W_mu(n) = U_mu(n) U_mu(n + mu) U_mu(n + 2 mu), every mu (one thread per (mu, n))
__global__ __launch_bounds__(256) void k_long(const double2* __restrict__ U, double2* __restrict__ W, FGeo g) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 4 * g.vol) return;
  const int mu = (int)(id / g.vol);
  const long n = id - (long)mu * g.vol;
  int c[4];
  coords(n, g, c);
  const double2* Um = U + 9 * (long)mu * g.vol;
  const long n1 = step(n, c, g, mu, 1);
  const long n2 = step(n, c, g, mu, 2);  // c + 2 < 2 L for L >= 2: one wrap suffices
  const M3 t = mul_nn(ld(mat(Um, n)), ld(mat(Um, n1)));
  st(mat(W + 9 * (long)mu * g.vol, n), mul_nn(t, ld(mat(Um, n2))));
}

inline unsigned blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t fatten_workspace_bytes(const int dims[4]) {
  const long vol = (long)dims[0] * dims[1] * dims[2] * dims[3];
  return (size_t)kFattenWsFields * vol * 9 * sizeof(double2);
}

hipError_t fatten_links(const int dims[4], const void* thin, double u0, void* fat, void* lng, void* ws,
                        hipStream_t st) {
  FGeo g;
  for (int i = 0; i < 4; ++i) g.L[i] = dims[i];
  g.stride[0] = 1;
  for (int i = 1; i < 4; ++i) g.stride[i] = g.stride[i - 1] * dims[i - 1];
  g.vol = g.stride[3] * dims[3];
  const long n9 = 9 * g.vol;
  const double2* U = static_cast<const double2*>(thin);
  double2* Vf = static_cast<double2*>(fat);
  double2* W = static_cast<double2*>(lng);
  double2* w = static_cast<double2*>(ws);
  double2* P = w;             // wrap^+ of U_mu in one transverse direction
  double2* Mn = w + n9;       // wrap^-
  double2* X[4] = {w + 2 * n9, w + 3 * n9, w + 4 * n9, nullptr};  // 3-link staples per transverse direction
  double2* Y = w + 5 * n9;    // one 5-link staple field (outer rho, inner si)
  const double u2 = 1.0 / (u0 * u0), u4 = u2 * u2, u6 = u4 * u2;
  const double c1 = 5.0 / 8.0, c3 = u2 / 16.0, c5 = u4 / 64.0, c7 = u6 / 384.0, cl = -u4 / 16.0;

  for (int mu = 0; mu < 4; ++mu) {
    const double2* Um = U + (long)mu * n9;
    double2* Vm = Vf + (long)mu * n9;
    int others[3], k = 0;
    for (int d = 0; d < 4; ++d)
      if (d != mu) others[k++] = d;
    hipLaunchKernelGGL(k_scale, dim3(blocks(n9)), dim3(256), 0, st, Um, Vm, c1, n9);
    for (int a = 0; a < 3; ++a) {
      const int nu = others[a];
      hipLaunchKernelGGL(k_wrap, dim3(blocks(g.vol)), dim3(256), 0, st, U, Um, P, 1.0, 0, (double2*)nullptr, 0.0,
                         mu, nu, 1, g);
      hipLaunchKernelGGL(k_wrap, dim3(blocks(g.vol)), dim3(256), 0, st, U, Um, Mn, 1.0, 0, (double2*)nullptr, 0.0,
                         mu, nu, 2, g);
      // Lepage: the same sign twice
      hipLaunchKernelGGL(k_wrap, dim3(blocks(g.vol)), dim3(256), 0, st, U, (const double2*)P, Vm, cl, 1,
                         (double2*)nullptr, 0.0, mu, nu, 1, g);
      hipLaunchKernelGGL(k_wrap, dim3(blocks(g.vol)), dim3(256), 0, st, U, (const double2*)Mn, Vm, cl, 1,
                         (double2*)nullptr, 0.0, mu, nu, 2, g);
      hipLaunchKernelGGL(k_staple_sum, dim3(blocks(n9)), dim3(256), 0, st, (const double2*)P, (const double2*)Mn,
                         X[a], Vm, c3, n9);
    }
    for (int a = 0; a < 3; ++a)      // outer rho
      for (int b = 0; b < 3; ++b) {  // inner si
        if (a == b) continue;
        const int rho = others[a], third = others[3 - a - b];
        // Y = (wrap_rho^+ + wrap_rho^-)(X_si), V += c5 Y
        hipLaunchKernelGGL(k_wrap, dim3(blocks(g.vol)), dim3(256), 0, st, U, (const double2*)X[b], Y, 1.0, 0, Vm,
                           c5, mu, rho, 3, g);
        // V += c7 (wrap_third^+ + wrap_third^-)(Y)
        hipLaunchKernelGGL(k_wrap, dim3(blocks(g.vol)), dim3(256), 0, st, U, (const double2*)Y, Vm, c7, 1,
                           (double2*)nullptr, 0.0, mu, third, 3, g);
      }
  }
  hipLaunchKernelGGL(k_long, dim3(blocks(4 * g.vol)), dim3(256), 0, st, U, W, g);
  return hipGetLastError();
}

}  // namespace stag
