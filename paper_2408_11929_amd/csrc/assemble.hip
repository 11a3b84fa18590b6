// P1 assembly of the impedance Helmholtz operator (eq. (1)) and of the strip
// matrices of the sweeping preconditioners (Sec. 2, Fig. 1; eq. (4) on the
// artificial sides), directly into the layouts the solver kernels read.
//
// Mesh: node (i, j) at (i h, j h), index p = j n + i; every cell is cut by its
// "/" diagonal into T_lo = {(i,j),(i+1,j),(i+1,j+1)} and
// T_up = {(i,j),(i,j+1),(i+1,j+1)}, both right isosceles with the right angle
// at the middle vertex as listed.  For such a triangle with legs h the P1
// stiffness matrix is 1/2 [[1,-1,0],[-1,2,-1],[0,-1,1]] and the mass matrix
// h^2/24 [[2,1,1],[1,2,1],[1,1,2]]; an edge of length h carries the impedance
// form -i k h/6 [[2,1],[1,2]].  A node couples to the 7-point "/" stencil
// (offsets 0, +-1, +-n, +-(n+1)).
#include <cstdlib>

#include <algorithm>

#include "hh_internal.h"

namespace hh {

namespace {

// Stencil slot of neighbour offset (di, dj), dj*n + di in {-n-1,-n,-1,0,1,n,n+1}.
__device__ __forceinline__ int slot_of(int di, int dj) {
  // (-1,-1)->0 (0,-1)->1 (-1,0)->2 (0,0)->3 (1,0)->4 (0,1)->5 (1,1)->6
  return dj == -1 ? (di == -1 ? 0 : 1) : (dj == 0 ? 3 + di : (di == 0 ? 5 : 6));
}

// Wave number at the sample height y = P / (6 (n-1)) of a layered medium.
__device__ __forceinline__ double wave_number(long long P, int n, int L, const double* c,
                                              double omega) {
  long long l = (P * (long long)L) / (6LL * (n - 1));
  if (l > L - 1) l = L - 1;
  return omega / c[l];
}

// Wave numbers of the triangles and edges (eq. (1), k = omega / c): from the
// layer table at the sample heights, or read from the tables a speed field
// was sampled into (Medium::kt, kv, kh).
__device__ __forceinline__ double k_triangle(const Medium& m, int n, int ci, int cj, int t) {
  if (m.kt) return m.kt[2 * ((long long)cj * (n - 1) + ci) + t];
  return wave_number(6LL * cj + (t == 0 ? 2 : 4), n, m.L, m.c, m.omega);
}
// edge (i, j) - (i + 1, j)
__device__ __forceinline__ double k_hedge(const Medium& m, int n, int i, int j) {
  if (m.kh) return m.kh[(long long)j * (n - 1) + i];
  return wave_number(6LL * j, n, m.L, m.c, m.omega);
}
// edge (i, j) - (i, j + 1)
__device__ __forceinline__ double k_vedge(const Medium& m, int n, int i, int j) {
  if (m.kv) return m.kv[(long long)j * n + i];
  return wave_number(6LL * j + 3, n, m.L, m.c, m.omega);
}

// The P1 stiffness part of row (i, j) over the window's cells.
__device__ void stiffness_stencil(int i, int j, int n, int cx0, int cx1, int cy0, int cy1,
                                  c128 out[7]) {
  const double Ks[3][3] = {{0.5, -0.5, 0.0}, {-0.5, 1.0, -0.5}, {0.0, -0.5, 0.5}};
  for (int cj = j - 1; cj <= j; ++cj) {
    if (cj < cy0 || cj >= cy1) continue;
    for (int ci = i - 1; ci <= i; ++ci) {
      if (ci < cx0 || ci >= cx1) continue;
      for (int t = 0; t < 2; ++t) {
        int vx[3], vy[3];
        vx[0] = ci; vy[0] = cj;
        if (t == 0) { vx[1] = ci + 1; vy[1] = cj; }
        else { vx[1] = ci; vy[1] = cj + 1; }
        vx[2] = ci + 1; vy[2] = cj + 1;
        int a = -1;
        for (int v = 0; v < 3; ++v)
          if (vx[v] == i && vy[v] == j) a = v;
        if (a < 0) continue;
        for (int b = 0; b < 3; ++b) out[slot_of(vx[b] - i, vy[b] - j)].re += Ks[a][b];
      }
    }
  }
}

// wave number at node (i, j) (five-point scheme): the sampled field, or the
// layer of the node's height y = 6 j / (6 (n-1))
__device__ __forceinline__ double k_node(const Medium& m, int n, int i, int j) {
  if (m.kn) return m.kn[(long long)j * n + i];
  return wave_number(6LL * j, n, m.L, m.c, m.omega);
}

// 7-point stencil of row (i, j) of the operator assembled over the cells of the
// window [cx0, cx1) x [cy0, cy1) with the impedance edge form on all four
// window sides.  mass_only: unit-weight mass matrix (for the load vector).
// Five-point scheme (md.fd5): the P1 stiffness of the window (on this mesh the
// five-point Laplacian in the scaling h^2 w) minus h^2 k^2 w on the diagonal
// and i h k on the window's boundary nodes, w = 1, 1/2 on a window side, 1/4 at
// a window corner (mass_only: h^2 w on the diagonal).
__device__ void node_stencil(int i, int j, int n, int cx0, int cx1, int cy0, int cy1,
                             const Medium& md, bool mass_only, c128 out[7]) {
  const double h = 1.0 / (n - 1);
  for (int d = 0; d < 7; ++d) out[d] = mk(0.0, 0.0);
  if (md.fd5) {
    const double wx = (i == cx0 || i == cx1) ? 0.5 : 1.0, wy = (j == cy0 || j == cy1) ? 0.5 : 1.0;
    const double w = wx * wy;
    if (mass_only) {
      out[3].re = h * h * w;
      return;
    }
    stiffness_stencil(i, j, n, cx0, cx1, cy0, cy1, out);
    const double k = k_node(md, n, i, j);
    out[3].re -= h * h * k * k * w;
    if (i == cx0 || i == cx1 || j == cy0 || j == cy1) out[3].im -= h * k;
    return;
  }
  const double Ks[3][3] = {{0.5, -0.5, 0.0}, {-0.5, 1.0, -0.5}, {0.0, -0.5, 0.5}};
  const double m0 = h * h / 24.0;
  // the four cells that contain node (i, j)
  for (int cj = j - 1; cj <= j; ++cj) {
    if (cj < cy0 || cj >= cy1) continue;
    for (int ci = i - 1; ci <= i; ++ci) {
      if (ci < cx0 || ci >= cx1) continue;
      for (int t = 0; t < 2; ++t) {
        int vx[3], vy[3];
        vx[0] = ci; vy[0] = cj;
        if (t == 0) { vx[1] = ci + 1; vy[1] = cj; }      // T_lo
        else { vx[1] = ci; vy[1] = cj + 1; }             // T_up
        vx[2] = ci + 1; vy[2] = cj + 1;
        int a = -1;
        for (int v = 0; v < 3; ++v)
          if (vx[v] == i && vy[v] == j) a = v;
        if (a < 0) continue;
        double k = mass_only ? 1.0 : k_triangle(md, n, ci, cj, t);
        double k2 = mass_only ? 1.0 : k * k;
        for (int b = 0; b < 3; ++b) {
          double mab = m0 * (a == b ? 2.0 : 1.0);
          double val = (mass_only ? 0.0 : Ks[a][b]) - (mass_only ? -mab : k2 * mab);
          int s = slot_of(vx[b] - i, vy[b] - j);
          out[s].re += val;
        }
      }
    }
  }
  if (mass_only) return;
  // impedance edges on the window sides
  const double e0 = h / 6.0;
  auto edge = [&](int bi, int bj, double k) {
    out[3].im -= k * e0 * 2.0;
    out[slot_of(bi - i, bj - j)].im -= k * e0;
  };
  if (j == cy0 || j == cy1) {            // bottom / top side
    if (i >= cx0 && i <= cx1) {
      if (i - 1 >= cx0) edge(i - 1, j, k_hedge(md, n, i - 1, j));
      if (i + 1 <= cx1) edge(i + 1, j, k_hedge(md, n, i, j));
    }
  }
  if (i == cx0 || i == cx1) {            // left / right side
    if (j >= cy0 && j <= cy1) {
      if (j - 1 >= cy0) edge(i, j - 1, k_vedge(md, n, i, j - 1));
      if (j + 1 <= cy1) edge(i, j + 1, k_vedge(md, n, i, j));
    }
  }
}

__global__ void k_assemble(int n, Medium md, c128* __restrict__ A) {
  long long nn = (long long)n * n;
  long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= nn) return;
  int i = (int)(p % n), j = (int)(p / n);
  c128 st[7];
  node_stencil(i, j, n, 0, n - 1, 0, n - 1, md, false, st);
  A[p] = st[3];
  A[nn + p] = st[4];
  A[2 * nn + p] = st[5];
  A[3 * nn + p] = st[6];
}

__global__ void k_load_vector(int n, int nvec, const c128* __restrict__ f, c128* __restrict__ b,
                              int fd5) {
  long long nn = (long long)n * n;
  long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= nn) return;
  int i = (int)(p % n), j = (int)(p / n);
  c128 st[7];
  Medium md{};
  md.fd5 = fd5;
  node_stencil(i, j, n, 0, n - 1, 0, n - 1, md, true, st);
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  for (int v = 0; v < nvec; ++v) {
    const c128* fv = f + v * nn;
    c128 acc = mk(0.0, 0.0);
    for (int d = 0; d < 7; ++d) {
      int ii = i + di[d], jj = j + dj[d];
      if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
      c128 fq = fv[(long long)jj * n + ii];
      acc.re -= st[d].re * fq.re;
      acc.im -= st[d].re * fq.im;
    }
    b[v * nn + p] = acc;
  }
}

// Fill the band storage of every strip: element (q, q') of A_s at column q',
// position kv + q - q' (kv = 2 kl), and the transmission stencils
// (A_s - A) on the interface rows.  grid.y = strip index.
// With redo given, only the strips marked 2 there are packed, and their
// transmission stencils (unchanged) are left alone.
template <class T>
__global__ void k_pack_strips(int n, Medium md,
                              const StripDesc* __restrict__ strips, cx<T>* __restrict__ band,
                              cx<T>* __restrict__ tr, const int* __restrict__ redo) {
  if (redo && redo[blockIdx.y] != 2) return;
  const StripDesc sd = strips[blockIdx.y];
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= sd.ns) return;
  const int kv = 2 * sd.kl;
  cx<T>* ab = band + sd.band_off;
  if (q >= sd.nr) {  // identity rows past the strip's unknowns
    if (band) ab[(long long)q * sd.ldab + kv] = mk((T)1, (T)0);
    return;
  }
  int l = q / sd.w, t = q - l * sd.w;
  int i, j, cx0, cx1, cy0, cy1;
  if (sd.dir == 0) {
    i = sd.a + t; j = l;
    cx0 = sd.a; cx1 = sd.a + sd.w - 1; cy0 = 0; cy1 = n - 1;
  } else {
    i = l; j = sd.a + t;
    cx0 = 0; cx1 = n - 1; cy0 = sd.a; cy1 = sd.a + sd.w - 1;
  }
  c128 st[7];
  node_stencil(i, j, n, cx0, cx1, cy0, cy1, md, false, st);
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  for (int d = 0; d < 7 && band; ++d) {  // band == nullptr: the transmission data only
    if (st[d].re == 0.0 && st[d].im == 0.0) continue;
    int ii = i + di[d], jj = j + dj[d];
    int qq = sd.dir == 0 ? jj * sd.w + (ii - sd.a) : ii * sd.w + (jj - sd.a);
    ab[(long long)qq * sd.ldab + kv + q - qq] = mk((T)st[d].re, (T)st[d].im);
  }
  bool side1 = (t == 0 && sd.has1 && !redo), side2 = (t == sd.w - 1 && sd.has2 && !redo);
  if (side1 || side2) {
    c128 g[7];
    node_stencil(i, j, n, 0, n - 1, 0, n - 1, md, false, g);
    cx<T>* out = tr + (side1 ? sd.tr1_off : sd.tr2_off) + 7LL * l;
    for (int d = 0; d < 7; ++d) out[d] = mk((T)(st[d].re - g[d].re), (T)(st[d].im - g[d].im));
  }
}

// Sub-blocks of the strips (recursive strip solves): the operator of the
// sub-block's rectangle with the impedance condition on all four sides, in
// the sub-block's order (orient 0: q' = L w + T, orient 1: q' = T len + L,
// L = line along the strip - c0, T = across), band-packed like a strip; and
// on its interface lines the transmission coefficients (A_{s,t} - A_s) of
// the seven stencil neighbours, node T at tr + tr{1,2}_off + 7 T.
// grid = (ns blocks, sub-blocks).
template <class T>
__global__ void k_pack_sub(int n, Medium md, const StripDesc* __restrict__ subs,
                           cx<T>* __restrict__ band, cx<T>* __restrict__ tr) {
  const StripDesc sd = subs[blockIdx.y];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= sd.ns) return;
  const int w = sd.w, len = sd.len;
  int L, Tt;
  if (sd.orient == 0) {
    L = q / w;
    Tt = q - L * w;
  } else {
    Tt = q / len;
    L = q - Tt * len;
  }
  const int l = sd.c0 + L;
  int i, j, cx0, cx1, cy0, cy1;
  if (sd.dir == 0) {
    i = sd.a + Tt; j = l;
    cx0 = sd.a; cx1 = sd.a + w - 1; cy0 = sd.c0; cy1 = sd.c0 + len - 1;
  } else {
    i = l; j = sd.a + Tt;
    cx0 = sd.c0; cx1 = sd.c0 + len - 1; cy0 = sd.a; cy1 = sd.a + w - 1;
  }
  c128 st[7];
  node_stencil(i, j, n, cx0, cx1, cy0, cy1, md, false, st);
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  const int kv = 2 * sd.kl;
  cx<T>* ab = band + sd.band_off;
  for (int d = 0; d < 7; ++d) {
    if (st[d].re == 0.0 && st[d].im == 0.0) continue;
    const int ii = i + di[d], jj = j + dj[d];
    const int T2 = sd.dir == 0 ? ii - sd.a : jj - sd.a;
    const int L2 = (sd.dir == 0 ? jj : ii) - sd.c0;
    const int qq = sd.orient == 0 ? L2 * w + T2 : T2 * len + L2;
    ab[(long long)qq * sd.ldab + kv + q - qq] = mk((T)st[d].re, (T)st[d].im);
  }
  const bool side1 = L == 0 && sd.has1, side2 = L == len - 1 && sd.has2;
  if (side1 || side2) {
    c128 g[7];
    if (sd.dir == 0)
      node_stencil(i, j, n, sd.a, sd.a + w - 1, 0, n - 1, md, false, g);
    else
      node_stencil(i, j, n, 0, n - 1, sd.a, sd.a + w - 1, md, false, g);
    cx<T>* out = tr + (side1 ? sd.tr1_off : sd.tr2_off) + 7LL * Tt;
    for (int d = 0; d < 7; ++d) out[d] = mk((T)(st[d].re - g[d].re), (T)(st[d].im - g[d].im));
  }
}

// Zeroes the band of every strip marked 2 in redo.  grid.y = strip index.
template <class T>
__global__ void k_zero_marked(const StripDesc* __restrict__ strips, cx<T>* __restrict__ band,
                              const int* __restrict__ redo) {
  if (redo[blockIdx.y] != 2) return;
  const StripDesc sd = strips[blockIdx.y];
  const long long ne = (long long)sd.ns * sd.ldab;
  cx<T>* ab = band + sd.band_off;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
       e += (long long)gridDim.x * blockDim.x)
    ab[e] = mk((T)0, (T)0);
}

}  // namespace

Medium medium_of(const hh_problem* pb) {
  Medium m{};
  m.omega = pb->omega;
  m.L = (int)pb->c.size();
  m.c = pb->d_c;
  m.kt = pb->d_kt;
  m.kv = pb->d_kv;
  m.kh = pb->d_kh;
  m.kn = pb->d_kn;
  m.fd5 = pb->scheme == HH_SCHEME_FD5;
  return m;
}

void launch_assemble(int n, const Medium& md, c128* d_A, hipStream_t st) {
  long long nn = (long long)n * n;
  int bs = 256;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((nn + bs - 1) / bs)), dim3(bs), 0, st, n, md, d_A);
  HH_HIP(hipGetLastError());
}

void launch_load_vector(int n, int nvec, const c128* f, c128* b, hipStream_t st, int fd5) {
  long long nn = (long long)n * n;
  int bs = 256;
  hipLaunchKernelGGL(k_load_vector, dim3((unsigned)((nn + bs - 1) / bs)), dim3(bs), 0, st, n,
                     nvec, f, b, fd5);
  HH_HIP(hipGetLastError());
}

void launch_pack_strips(const hh_problem* pb, hipStream_t st) {
  const FactorSet& fs = pb->fs;
  size_t esz = fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
  HH_HIP(hipMemsetAsync(fs.band, 0, fs.band_elems * esz, st));
  HH_HIP(hipMemsetAsync(fs.tr, 0, fs.tr_elems * esz, st));
  int bs = 256;
  if (fs.nsub > 1) {
    // recursive strip solves: the outer strips give their transmission data
    // only, the sub-blocks their matrices and inner transmission data
    const dim3 go((unsigned)((fs.max_ns + bs - 1) / bs), (unsigned)fs.first_sub);
    int ns_sub = 0;
    for (size_t u = fs.first_sub; u < fs.strips.size(); ++u) ns_sub = std::max(ns_sub, fs.strips[u].ns);
    const dim3 gs((unsigned)((ns_sub + bs - 1) / bs), (unsigned)(fs.strips.size() - fs.first_sub));
    if (fs.precision == HH_FP64) {
      hipLaunchKernelGGL(k_pack_strips<double>, go, dim3(bs), 0, st, pb->n, medium_of(pb),
                         fs.d_strips, (c128*)nullptr, (c128*)fs.tr, (const int*)nullptr);
      hipLaunchKernelGGL(k_pack_sub<double>, gs, dim3(bs), 0, st, pb->n, medium_of(pb),
                         fs.d_strips + fs.first_sub, (c128*)fs.band, (c128*)fs.tr);
    } else {
      hipLaunchKernelGGL(k_pack_strips<float>, go, dim3(bs), 0, st, pb->n, medium_of(pb),
                         fs.d_strips, (c64*)nullptr, (c64*)fs.tr, (const int*)nullptr);
      hipLaunchKernelGGL(k_pack_sub<float>, gs, dim3(bs), 0, st, pb->n, medium_of(pb),
                         fs.d_strips + fs.first_sub, (c64*)fs.band, (c64*)fs.tr);
    }
    HH_HIP(hipGetLastError());
    return;
  }
  dim3 grid((unsigned)((fs.max_ns + bs - 1) / bs), (unsigned)fs.strips.size());
  if (fs.precision == HH_FP64)
    hipLaunchKernelGGL(k_pack_strips<double>, grid, dim3(bs), 0, st, pb->n, medium_of(pb),
                       fs.d_strips, (c128*)fs.band, (c128*)fs.tr,
                       (const int*)nullptr);
  else
    hipLaunchKernelGGL(k_pack_strips<float>, grid, dim3(bs), 0, st, pb->n, medium_of(pb),
                       fs.d_strips, (c64*)fs.band, (c64*)fs.tr,
                       (const int*)nullptr);
  HH_HIP(hipGetLastError());
}

void launch_repack_marked(const hh_problem* pb, hipStream_t st) {
  const FactorSet& fs = pb->fs;
  const int bs = 256;
  const dim3 zgrid(64, (unsigned)fs.strips.size());
  const dim3 grid((unsigned)((fs.max_ns + bs - 1) / bs), (unsigned)fs.strips.size());
  if (fs.precision == HH_FP64) {
    hipLaunchKernelGGL(k_zero_marked<double>, zgrid, dim3(bs), 0, st, fs.d_strips,
                       (c128*)fs.band, (const int*)fs.d_pflag);
    hipLaunchKernelGGL(k_pack_strips<double>, grid, dim3(bs), 0, st, pb->n, medium_of(pb),
                       fs.d_strips, (c128*)fs.band, (c128*)fs.tr,
                       (const int*)fs.d_pflag);
  } else {
    hipLaunchKernelGGL(k_zero_marked<float>, zgrid, dim3(bs), 0, st, fs.d_strips,
                       (c64*)fs.band, (const int*)fs.d_pflag);
    hipLaunchKernelGGL(k_pack_strips<float>, grid, dim3(bs), 0, st, pb->n, medium_of(pb),
                       fs.d_strips, (c64*)fs.band, (c64*)fs.tr,
                       (const int*)fs.d_pflag);
  }
  HH_HIP(hipGetLastError());
}

bool lu_interchanging_only() {
  const char* env = std::getenv("HH_LU_INTERCHANGE");
  return env && std::atoi(env) > 0;
}

}  // namespace hh
