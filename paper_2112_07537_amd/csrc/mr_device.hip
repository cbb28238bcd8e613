// HIP kernels (gfx950) of the multiresolution block-octree hot path.
//
// Method: Gillis & van Rees, MURPHY (arXiv 2112.07537).  Filter constants are
// those of the supplementary filter-bank tables (non-lifted 2.0/4.0/6.0 and
// lifted 2.2/4.2/6.2, acting on interleaved scaling/detail coefficients).
// Everything here is short stencil or filter work on blocks, so it is written
// for the memory system (coalesced block rows, LDS planes, register columns),
// not for the matrix cores.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include <hip/hip_ext.h>

#include "mr_internal.h"

namespace mr {

// Optional events recorded by the runtime exactly at the start and end of
// the next launch (hipExtLaunchKernel), used by the kernel timers.
static hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
void set_launch_events(hipEvent_t a, hipEvent_t b) {
  g_ev_start = a;
  g_ev_stop = b;
}
#define MR_LAUNCH(kernel, grid, block, lds, stream, ...)                                  \
  do {                                                                                    \
    if (g_ev_start)                                                                       \
      hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, g_ev_start, g_ev_stop, 0,   \
                            __VA_ARGS__);                                                 \
    else                                                                                  \
      hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                  \
  } while (0)

// ------------------------------------------------------------------ filters
// Deslauriers-Dubuc prediction of order N (K^s at the scaling positions):
// odd fine value 2k+1 = sum_j w[j - J0] * lambda_{k+j}, j in [1-N/2, N/2].
template <int N> struct DD;
template <> struct DD<2> {
  static constexpr int J0 = 0;
  __device__ static constexpr double w(int i) { return 0.5; }
};
template <> struct DD<4> {
  static constexpr int J0 = -1;
  __device__ static constexpr double w(int i) {
    return (i == 0 || i == 3) ? -1.0 / 16.0 : 9.0 / 16.0;
  }
};
template <> struct DD<6> {
  static constexpr int J0 = -2;
  __device__ static constexpr double w(int i) {
    return (i == 0 || i == 5) ? 3.0 / 256.0 : ((i == 1 || i == 4) ? -25.0 / 256.0 : 75.0 / 128.0);
  }
};

// Analysis H^a (even positions), reach HR, and G^a (odd positions), reach N-1.
template <int N, int NT> struct Ha;
template <int N> struct Ha<N, 0> {
  static constexpr int R = 0;
  __device__ static constexpr double c(int o) { return o == 0 ? 1.0 : 0.0; }
};
template <> struct Ha<2, 2> {
  static constexpr int R = 2;
  __device__ static constexpr double c(int o) {
    return o == 0 ? 0.75 : ((o == 1 || o == -1) ? 0.25 : -0.125);
  }
};
template <> struct Ha<4, 2> {
  static constexpr int R = 4;
  __device__ static constexpr double c(int o) {
    return o == 0 ? 23.0 / 32.0
         : (o == 1 || o == -1) ? 0.25
         : (o == 2 || o == -2) ? -0.125
         : (o == 4 || o == -4) ? 1.0 / 64.0 : 0.0;
  }
};
template <> struct Ha<6, 2> {
  static constexpr int R = 6;
  __device__ static constexpr double c(int o) {
    return o == 0 ? 181.0 / 256.0
         : (o == 1 || o == -1) ? 0.25
         : (o == 2 || o == -2) ? -125.0 / 1024.0
         : (o == 4 || o == -4) ? 11.0 / 512.0
         : (o == 6 || o == -6) ? -3.0 / 1024.0 : 0.0;
  }
};
template <int N> struct Ga {
  static constexpr int R = N - 1;
  // centre 1, odd offsets minus the DD weights, even offsets 0
  __device__ static constexpr double c(int o) {
    return o == 0 ? 1.0 : ((o & 1) ? -DD<N>::w((o + 1) / 2 - DD<N>::J0) : 0.0);
  }
};
// Synthesis J^s (even) and K^s (odd) of the interleaved layout.
template <int N, int NT> struct Js;
template <int N> struct Js<N, 0> {
  static constexpr int R = 0;
  __device__ static constexpr double c(int o) { return o == 0 ? 1.0 : 0.0; }
};
template <int N> struct Js<N, 2> {
  static constexpr int R = 1;
  __device__ static constexpr double c(int o) { return o == 0 ? 1.0 : -0.25; }
};
template <int N, int NT> struct Ks;
template <int N> struct Ks<N, 0> {
  static constexpr int R = N - 1;
  __device__ static constexpr double c(int o) {
    return o == 0 ? 1.0 : ((o & 1) ? DD<N>::w((o + 1) / 2 - DD<N>::J0) : 0.0);
  }
};
template <int N> struct Ks<N, 2> {
  static constexpr int R = N;
  // odd offsets: DD weights; even offsets: -1/4 * (DD-weighted J^s neighbours)
  __device__ static constexpr double c(int o) {
    if (o & 1) return DD<N>::w((o + 1) / 2 - DD<N>::J0);
    // f[2k+1] gets -1/4 (gamma_{k-1+j} + gamma_{k+j}) through each lambda_{k+j}
    // used by the prediction; collect the weight of gamma at offset o.
    double s = (o == 0) ? 1.0 : 0.0;
    for (int i = 0; i < N; ++i) {
      int j = i + DD<N>::J0;           // lambda_{k+j} at offset 2j-1
      int lo = 2 * j - 2, hi = 2 * j;  // gammas around it at offsets 2j-2, 2j
      if (o == lo || o == hi) s += -0.25 * DD<N>::w(i);
    }
    return s;
  }
};

// ------------------------------------------------------------ index helpers
__device__ __forceinline__ int floordiv(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__device__ __forceinline__ int wrapi(int a, int w) {
  int r = a % w;
  return r < 0 ? r + w : r;
}

// floor(a / b) for 0 <= a < 2^20 and 1 <= b < 2^11 through the FP32
// reciprocal: (a + 1/2) / b lies at least 1/(2b) away from an integer, and
// the relative error of the product (one rounding of a + 1/2, the
// reciprocal's 1 ulp, one rounding of the product) stays below 2^-21, i.e.
// below 1/(2b) in absolute terms for a below 2^20.
__device__ __forceinline__ int div_small(int a, int b) {
  return int((float(a) + 0.5f) * __builtin_amdgcn_rcpf(float(b)));
}

// Leaf id holding the level-(L+up) point q given relative to block m.
template <typename T>
__device__ __forceinline__ int owner_id(const DevGrid<T>& g, int m, int up, int qx, int qy, int qz) {
  const int h = g.nb >> 1;
  const int ax = (qx >> up) + h, ay = (qy >> up) + h, az = (qz >> up) + h;
  if ((unsigned)ax >= unsigned(4 * h) || (unsigned)ay >= unsigned(4 * h) ||
      (unsigned)az >= unsigned(4 * h)) {
    atomicAdd(g.err, 1);
    return -1;
  }
  const int cx = div_small(ax, h), cy = div_small(ay, h), cz = div_small(az, h);
  return g.cmap[m * 64 + (cz * 4 + cy) * 4 + cx];
}

// Value of block b's level-L field extended by its ghost layer: own points,
// same-level neighbours, or the cross-level patch of the region.
template <typename T>
__device__ __forceinline__ T ext_value(const DevGrid<T>& g, int b, int x, int y, int z) {
  const int nb = g.nb;
  const int rx = x < 0 ? 0 : (x < nb ? 1 : 2);
  const int ry = y < 0 ? 0 : (y < nb ? 1 : 2);
  const int rz = z < 0 ? 0 : (z < nb ? 1 : 2);
  const int r = rx + 3 * ry + 9 * rz;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  if (r == 13) return g.field[b * nb3 + ((int64_t)z * nb + y) * nb + x];
  const int64_t po = g.poff[(int64_t)b * 27 + r];
  if (po < 0) {
    const int cx = rx == 0 ? 0 : (rx == 1 ? 1 : 3);
    const int cy = ry == 0 ? 0 : (ry == 1 ? 1 : 3);
    const int cz = rz == 0 ? 0 : (rz == 1 ? 1 : 3);
    const int n = g.cmap[b * 64 + (cz * 4 + cy) * 4 + cx];
    return g.field[n * nb3 + ((int64_t)(z - (rz - 1) * nb) * nb + (y - (ry - 1) * nb)) * nb +
                   (x - (rx - 1) * nb)];
  }
  const int dw = g.dw;
  const int sx = rx == 1 ? nb : dw, sy = ry == 1 ? nb : dw;
  const int lx = rx == 0 ? -dw : (rx == 1 ? 0 : nb);
  const int ly = ry == 0 ? -dw : (ry == 1 ? 0 : nb);
  const int lz = rz == 0 ? -dw : (rz == 1 ? 0 : nb);
  return g.patch[po + ((int64_t)(z - lz) * sy + (y - ly)) * sx + (x - lx)];
}

// Owner-map cells of block m cached in LDS: leaf id, level, origin at its
// level.  Turns a sample lookup into LDS reads plus one global load.
struct CellTab {
  int32_t id[64], lev[64], ox[64], oy[64], oz[64];
};

template <typename T>
__device__ __forceinline__ void load_cells(const DevGrid<T>& g, int m, CellTab& ct) {
  const int t = threadIdx.x;
  if (t < 64) {
    const int id = g.cmap[m * 64 + t];
    ct.id[t] = id;
    ct.lev[t] = g.lev[id];
    ct.ox[t] = g.ijk[3 * id] * g.nb;
    ct.oy[t] = g.ijk[3 * id + 1] * g.nb;
    ct.oz[t] = g.ijk[3 * id + 2] * g.nb;
  }
}

__device__ __forceinline__ int wrap1(int X, int W) {
  X += (X < 0) ? W : 0;
  X -= (X >= W) ? W : 0;
  return X;
}

// Element index of the value of the leaf holding the level-L point p
// (relative to block m at level L, origin O), by injection, clamped into that
// leaf; *bad is set when p is outside the owner map or not on the leaf's grid.
// Branch-free, so a thread can issue several loads before waiting on any.
template <int NB>
__device__ __forceinline__ int64_t cell_index(const CellTab& ct, int L, int Ox, int Oy, int Oz,
                                              int px, int py, int pz, int& bad) {
  constexpr int H = NB / 2;
  unsigned ux = unsigned(px + H), uy = unsigned(py + H), uz = unsigned(pz + H);
  bad |= int(ux >= 4u * H) | int(uy >= 4u * H) | int(uz >= 4u * H);
  ux = min(ux, 4u * H - 1u);
  uy = min(uy, 4u * H - 1u);
  uz = min(uz, 4u * H - 1u);
  const int c = ((uz / H) * 4 + uy / H) * 4 + ux / H;
  const int W = NB << L;
  int X = wrap1(Ox + px, W), Y = wrap1(Oy + py, W), Z = wrap1(Oz + pz, W);
  const int l = ct.lev[c];
  bad |= int(l < L) & ((X | Y | Z) & 1);
  X = l > L ? (X << 1) : (l < L ? (X >> 1) : X);
  Y = l > L ? (Y << 1) : (l < L ? (Y >> 1) : Y);
  Z = l > L ? (Z << 1) : (l < L ? (Z >> 1) : Z);
  unsigned lx = unsigned(X - ct.ox[c]), ly = unsigned(Y - ct.oy[c]), lz = unsigned(Z - ct.oz[c]);
  bad |= int(lx >= unsigned(NB)) | int(ly >= unsigned(NB)) | int(lz >= unsigned(NB));
  lx = min(lx, unsigned(NB - 1));
  ly = min(ly, unsigned(NB - 1));
  lz = min(lz, unsigned(NB - 1));
  return (int64_t)ct.id[c] * (NB * NB * NB) + int((lz * NB + ly) * NB + lx);
}

// Flattened iteration over a 3D box [0,w0) x [0,w1) x [0,w2) with a fixed
// thread stride, carrying the coordinates incrementally (no divisions in the
// loop; the stride is decomposed once).
struct Iter3 {
  int x, y, z, w0, w1, sx, sy, sz;
  // start, step < 2^20 (thread index and workgroup size); w0, w1 >= 1 and
  // below 2^11 (box extents)
  __device__ __forceinline__ Iter3(int start, int step, int w0_, int w1_) : w0(w0_), w1(w1_) {
    int t = div_small(start, w0);
    x = start - t * w0;
    z = div_small(t, w1);
    y = t - z * w1;
    t = div_small(step, w0);
    sx = step - t * w0;
    sz = div_small(t, w1);
    sy = t - sz * w1;
  }
  __device__ __forceinline__ void advance() {
    x += sx;
    y += sy;
    z += sz;
    if (x >= w0) {
      x -= w0;
      ++y;
    }
    if (y >= w1) {
      y -= w1;
      ++z;
    }
  }
};

// XCD-aware item order: workgroup i runs on XCD i % 8; give each XCD one
// contiguous run of items (items are in Morton block order).
__device__ __forceinline__ int xcd_item(int i, int n) {
  if (n < 64) return i;
  const int q = n >> 3, r = n & 7, x = i & 7, k = i >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Affine address table of the 64 owner-map cells of a block for coarse
// samples: the level-(L-1) sample c (relative to the block's origin, i.e.
// the level-L point p = 2c) held by the leaf of cell k sits at element
//   base[k] + step[k] * (c_x + NB c_y + NB^2 c_z)
// of the field (step 1, 2 or 4 for a leaf one level coarser, at the same
// level, one level finer).  The periodic wrap is constant inside a cell,
// so it is folded into base.  The table depends on the tree only; it is
// built once per tree, one thread per (block, cell), and flags leaves
// outside L-1..L+1.
template <typename T, int NB>
__global__ void k_cell_tables(DevGrid<T> g, int64_t* base, int32_t* step, int n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * 64) return;
  const int m = int(i >> 6), t = int(i & 63);
  constexpr int H = NB / 2;
  const int L = g.lev[m];
  const int id = g.cmap[i];
  const int l = g.lev[id];
  const int W = NB << L;
  const int cc[3] = {t & 3, (t >> 2) & 3, t >> 4};
  int64_t b = (int64_t)id * (NB * NB * NB);
  int64_t mul = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int O = g.ijk[3 * m + a] * NB;
    const int X0 = O + (cc[a] - 1) * H;
    const int shift = X0 - wrap1(X0, W);
    const int o = g.ijk[3 * id + a] * NB;
    const int base_a = l == L ? (O - shift) - o : (l > L ? 2 * (O - shift) - o : (O - shift) / 2 - o);
    b += mul * base_a;
    mul *= NB;
  }
  base[i] = b;
  step[i] = l == L ? 2 : (l > L ? 4 : 1);
  if (l < L - 1 || l > L + 1) atomicAdd(g.err, 1);
}

// One workgroup per GItem.  S = coarse samples [cs2][cs1][cs0], T1 = refined
// along x [cs2][cs1][fs0], T2 = refined along y [cs2][fs1][fs0] (aliases S),
// then z is refined and written out.  Each refinement pass computes pairs of
// fine points (2c, 2c+1) from the samples c-N/2+1 .. c+N/2.
template <typename T, int N, int NT, int NB>
__global__ __launch_bounds__(256) void k_gview(DevGrid<T> g, const GItem* __restrict__ items) {
  extern __shared__ unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  __shared__ int64_t cbase[64];
  __shared__ int32_t cstep[64];
  __shared__ uint8_t acell[3][32];
  __shared__ int64_t roff[27];
  constexpr int J0 = 1 - N / 2;   // first DD tap offset
  constexpr int HN = N / 2 - 1;   // index of sample c inside the window
  const GItem it = items[xcd_item(blockIdx.x, gridDim.x)];
  const int m = it.blk;
  const int tid = threadIdx.x, nt = blockDim.x;
  int clo[3], cs[3], fs[3], np[3], e[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int p0 = it.lo[a] >> 1, p1 = (it.hi[a] - 1) >> 1;  // first / last pair
    clo[a] = p0 + J0;
    cs[a] = p1 - p0 + N;
    fs[a] = it.hi[a] - it.lo[a];
    np[a] = p1 - p0 + 1;
    e[a] = it.lo[a] & 1;   // 1: the first pair's even point is outside the box
  }
  if (tid < 64) {
    cbase[tid] = g.cbase[(int64_t)m * 64 + tid];
    cstep[tid] = g.cstep[(int64_t)m * 64 + tid];
  }
  if (tid >= 128 && tid < 128 + 27) roff[tid - 128] = g.poff[(int64_t)m * 27 + tid - 128];
  if (tid < 96) {
    const int a = tid >> 5, i = tid & 31;
    if (i < cs[a]) acell[a][i] = uint8_t((2 * (clo[a] + i) + NB / 2) / (NB / 2));
  }
  T* T1 = lds;
  T* S = T1 + fs[0] * cs[1] * cs[2];
  T* T2 = S;
  __syncthreads();
  {
    // one round of loads covers a side item's samples; slots past the end
    // skip their work (whole waves at a time)
    constexpr int U = 16;
    const int n = cs[0] * cs[1] * cs[2];
    const int lin0 = clo[0] + NB * clo[1] + NB * NB * clo[2];
    Iter3 q(tid, nt, cs[0], cs[1]);
    for (int i0 = tid; i0 < n; i0 += U * nt) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (i0 + u * nt < n) {
          const int k = (acell[2][q.z] * 4 + acell[1][q.y]) * 4 + acell[0][q.x];
          // sample offset from the cell's base: step times the F-frame
          // linear index (|index| < 2^23, step <= 4)
          const int lin = lin0 + q.x + NB * q.y + NB * NB * q.z;
          v[u] = g.field[cbase[k] + __mul24(cstep[k], lin)];
        }
        q.advance();
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * nt < n) S[i0 + u * nt] = v[u];
    }
  }
  __syncthreads();
  {  // x: pairs j along x, rows (y, z) of samples
    const int n = np[0] * cs[1] * cs[2];
    Iter3 q(tid, nt, np[0], cs[1]);
    for (int i = tid; i < n; i += nt, q.advance()) {
      const int r = q.z * cs[1] + q.y;
      const T* src = S + r * cs[0] + q.x;
      T od = T(0);
#pragma unroll
      for (int k = 0; k < N; ++k) od += T(DD<N>::w(k)) * src[k];
      const int x0 = 2 * q.x - e[0];
      T* dst = T1 + r * fs[0];
      if (x0 >= 0) dst[x0] = src[HN];
      if (x0 + 1 < fs[0]) dst[x0 + 1] = od;
    }
  }
  __syncthreads();
  // y and z passes by line segments: a work unit refines K consecutive
  // pairs of one line from a register window of N + K - 1 samples (line
  // index fastest across threads, so neighbouring lanes read neighbouring
  // LDS words)
  constexpr int K = 4;
  auto segment = [&](const T* src, int ss, int j0, int jn, auto&& put) {
    T win[N + K - 1];
#pragma unroll
    for (int k = 0; k < N + K - 1; ++k) win[k] = k < N - 1 + jn ? src[(j0 + k) * ss] : T(0);
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if (q < jn) {
        T od = T(0);
#pragma unroll
        for (int k = 0; k < N; ++k) od += T(DD<N>::w(k)) * win[q + k];
        put(j0 + q, win[q + HN], od);
      }
    }
  };
  {  // y: lines (x, z) of T1, pairs along y
    const int nl = fs[0] * cs[2], nseg = (np[1] + K - 1) / K;
    int l = tid, sg = 0;
    while (l >= nl) { l -= nl; ++sg; }
    for (int u = tid; u < nl * nseg; u += nt) {
      const int qx = l % fs[0], qz = l / fs[0];
      const T* src = T1 + qz * cs[1] * fs[0] + qx;
      T* dst = T2 + qz * fs[1] * fs[0] + qx;
      const int j0 = sg * K, jn = min(K, np[1] - j0);
      segment(src, fs[0], j0, jn, [&](int j, T ev, T od) {
        const int y0 = 2 * j - e[1];
        if (y0 >= 0) dst[y0 * fs[0]] = ev;
        if (y0 + 1 < fs[1]) dst[(y0 + 1) * fs[0]] = od;
      });
      l += nt;
      while (l >= nl) { l -= nl; ++sg; }
    }
  }
  __syncthreads();
  {  // z: lines (x, y) of T2, pairs along z, written out
    const int nl = fs[0] * fs[1], nseg = (np[2] + K - 1) / K;
    const int plane = fs[0] * fs[1];
    const int dw = g.dw;
    int l = tid, sg = 0;
    while (l >= nl) { l -= nl; ++sg; }
    for (int u = tid; u < nl * nseg; u += nt) {
      const int qx = l % fs[0], qy = l / fs[0];
      const int x = it.lo[0] + qx, y = it.lo[1] + qy;
      const T* src = T2 + l;
      const int j0 = sg * K, jn = min(K, np[2] - j0);
      {
        // region of the column and its place in that region's patch box
        // (depth dw on the axes outside the block); a pair never straddles
        // a region boundary in z (both are even)
        const int rx = x < 0 ? 0 : (x < NB ? 1 : 2);
        const int ry = y < 0 ? 0 : (y < NB ? 1 : 2);
        const int sx = rx == 1 ? NB : dw, sy = ry == 1 ? NB : dw;
        const int lxy = (y + (ry == 0 ? dw : (ry == 1 ? 0 : -NB))) * sx +
                        x + (rx == 0 ? dw : (rx == 1 ? 0 : -NB));
        segment(src, plane, j0, jn, [&](int j, T ev, T od) {
          const int z0 = it.lo[2] + 2 * j - e[2];
          const int rz = z0 < 0 ? 0 : (z0 < NB ? 1 : 2);
          const int r = rx + 3 * ry + 9 * rz;
          if ((it.rmask >> r) & 1) {
            const int lz = z0 + (rz == 0 ? dw : (rz == 1 ? 0 : -NB));
            T* dst = g.patch + roff[r] + lz * (sx * sy) + lxy;
            if (z0 >= it.lo[2]) dst[0] = ev;
            if (z0 + 1 < it.hi[2]) dst[sx * sy] = od;
          }
        });
      }
      l += nt;
      while (l >= nl) { l -= nl; ++sg; }
    }
  }
}

// --------------------------------------------------------- RHS + RK stage
// One workgroup per block, one thread per (x, y) column.  The column's z
// stencil lives in registers, the current plane (with its x/y halo) in LDS.
struct Desc {
  int64_t off;   // element offset such that value = buf[off + x + y*sy + z*sz]
  int32_t sy, sz;
  int32_t patch; // 1: patch buffer, 0: field
  int32_t pad;
};

template <typename T>
__device__ __forceinline__ void make_desc(const DevGrid<T>& g, int b, int r, Desc& d) {
  const int nb = g.nb;
  const int rx = r % 3, ry = (r / 3) % 3, rz = r / 9;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  if (r == 13) {
    d.off = b * nb3;
    d.sy = nb;
    d.sz = nb * nb;
    d.patch = 0;
    return;
  }
  const int64_t po = g.poff[(int64_t)b * 27 + r];
  if (po < 0) {
    const int cx = rx == 0 ? 0 : (rx == 1 ? 1 : 3);
    const int cy = ry == 0 ? 0 : (ry == 1 ? 1 : 3);
    const int cz = rz == 0 ? 0 : (rz == 1 ? 1 : 3);
    const int n = g.cmap[b * 64 + (cz * 4 + cy) * 4 + cx];
    d.off = n * nb3 - ((int64_t)(rx - 1) * nb + (int64_t)(ry - 1) * nb * nb +
                       (int64_t)(rz - 1) * nb * nb * nb);
    d.sy = nb;
    d.sz = nb * nb;
    d.patch = 0;
    return;
  }
  const int dw = g.dw;
  const int sx = rx == 1 ? nb : dw, sy = ry == 1 ? nb : dw;
  const int lx = rx == 0 ? -dw : (rx == 1 ? 0 : nb);
  const int ly = ry == 0 ? -dw : (ry == 1 ? 0 : nb);
  const int lz = rz == 0 ? -dw : (rz == 1 ? 0 : nb);
  d.sy = sx;
  d.sz = sx * sy;
  d.off = po - lx - (int64_t)ly * sx - (int64_t)lz * sx * sy;
  d.patch = 1;
}

// ------------------------------------------------------------ substitution
// Lattice of a substitution item along one axis: the coordinates a box
// point's chain of stencils can read, i.e. the even ones of [lo - R, hi + R)
// (nE of them, from e0) followed by the odd ones of [lo, hi) (nO, from o0),
// R = N - 1.  In this "combined" order the G^a taps of the odd point with
// odd index i (combined nE + i) are the even points with indices i .. i+N-1.
struct SubstAxis {
  int e0, o0, nE, nO, nL;
};

__host__ __device__ __forceinline__ SubstAxis subst_axis(int lo, int hi, int R) {
  SubstAxis a;
  const int s = lo - R;
  a.e0 = s + (s & 1);
  a.nE = (hi + R - a.e0 + 1) >> 1;
  a.o0 = lo | 1;
  a.nO = hi > a.o0 ? (hi - a.o0 + 1) >> 1 : 0;
  a.nL = a.nE + a.nO;
  return a;
}

// Sum over the N taps w_j = G^a(2j - R) of p[j * stride] (the odd offsets
// -R .. R of the one-axis filter, in a fixed order).
template <typename T, int N>
__device__ __forceinline__ T gtaps(const T* p, int stride) {
  T acc[2] = {T(0), T(0)};
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j & 1] += T(Ga<N>::c(2 * j - (N - 1))) * p[j * stride];
  return acc[0] + acc[1];
}

// fn(i0, i1, i2) over a box of extents n0 x n1 x n2, i0 fastest, spread over
// the workgroup.
template <typename Fn>
__device__ __forceinline__ void for_box(int n0, int n1, int n2, Fn fn) {
  const int n = n0 * n1 * n2;
  if (n == 0) return;
  Iter3 q(threadIdx.x, blockDim.x, n0, n1);
  for (int i = threadIdx.x; i < n; i += blockDim.x, q.advance()) fn(q.x, q.y, q.z);
}

// One workgroup per substitution item: a box of fine block F's slab points
// (section 2.3: a point of degree k, with k odd indices, gets minus the
// non-central taps of the tensor product of G^a over its odd axes; degree 1
// first, then 2, then 3, each reading the lower degrees' new values; 1D
// sign of section 2.2.4).
//
// The item stages F's ghost-filled values on the lattice of its box (per
// axis the even coordinates within N-1 of the box and the odd ones inside
// it, in the combined order above): F's own points, same-level neighbours'
// points and, in coarser regions, F's c->f patches, which hold the
// refinement of the samples from before the substitution (the patch launch
// runs first).  Each lattice point carries its slab flag from the owning
// block's slab table (bit lo | hi << 3 | parity << 6 set when a point with
// that front / back slab range membership and parity lies in one of the
// block's slabs).  Every flagged lattice point of degree 1 and then 2 is
// recomputed, and the box's points of degree 3; the tensor sums run as 1D
// passes (degree 2: along the second odd axis into a temporary, then the
// first; degree 3: z, y, then x), with the central term left out where the
// point itself would enter.  Finally the box's flagged points go to the field
// in natural order.
//
// Items run in any order and each writes only its own box (the host cuts a
// block's slabs into disjoint boxes), but reads points of other boxes, its
// own block's and its same-level neighbours'.  Every slab value a box point
// depends on is recomputed here from all-even points and points outside
// every slab, which no item writes; so whether a staged slab value was read
// before or after its own item wrote it never matters, and the result does
// not depend on the order of the items.  With 26-neighbour 2:1 balance no
// finer region lies within the widened box of a slab.
// a * b + c for non-negative operands below 2^24 (full-rate 24-bit multiply)
__device__ __forceinline__ int imad24(int a, int b, int c) { return int(__umul24(a, b)) + c; }

template <typename T, int N, int NT, int NB, int TPB>
__global__ __launch_bounds__(TPB) void k_subst(DevGrid<T> g, const GItem* __restrict__ items) {
  extern __shared__ unsigned char lds_raw[];
  // per region around F: element offset, from the start of the field, of
  // the point (0, 0, 0) of F's frame in the buffer that holds the region
  // (the field or the patch buffer: both are slices of one allocation or
  // separate allocations aligned to the element size), and the region's y
  // and z strides
  struct SDesc {
    int64_t off;
    int32_t sy, sz;
  };
  __shared__ SDesc desc[27];
  __shared__ uint32_t tab[27][16];  // slab tables of the blocks owning the
                                    // regions at F's level (zero otherwise)
  // per axis and combined lattice index: .x the coordinate relative to F;
  // .y the region's share of the region number (r = rx + 3 ry + 9 rz, bits
  // 0-4) plus, from bit 8, the point's front / back slab membership and
  // parity in the block holding it at bits a, 3 + a and 6 + a, so that the
  // three axes' .y add up to the region and the slab-table bit index
  __shared__ int2 lut[3][32];
  constexpr int R = N - 1;
  constexpr int FL = NT ? N : N - 1;        // front slab [0, FL)
  constexpr int BL = NT ? NB - N + 1 : NB - N + 2;   // back slab [BL, NB)
  const GItem it = items[xcd_item(blockIdx.x, gridDim.x)];
  const int F = it.blk;
  const int tid = threadIdx.x, nt = blockDim.x;
  const SubstAxis ax = subst_axis(it.lo[0], it.hi[0], R);
  const SubstAxis ay = subst_axis(it.lo[1], it.hi[1], R);
  const SubstAxis az = subst_axis(it.lo[2], it.hi[2], R);
  if (tid < 27) {
    Desc d;
    make_desc(g, F, tid, d);
    const int64_t pshift =
        (int64_t)(reinterpret_cast<uintptr_t>(g.patch) - reinterpret_cast<uintptr_t>(g.field)) /
        (int64_t)sizeof(T);
    desc[tid].off = d.off + (d.patch ? pshift : 0);
    desc[tid].sy = d.sy;
    desc[tid].sz = d.sz;
  }
  if (tid < 27 * 8) {
    const int r = tid >> 3, w = tid & 7;
    const int rx = r % 3, ry = (r / 3) % 3, rz = r / 9;
    const int cx = rx == 0 ? 0 : (rx == 1 ? 1 : 3);
    const int cy = ry == 0 ? 0 : (ry == 1 ? 1 : 3);
    const int cz = rz == 0 ? 0 : (rz == 1 ? 1 : 3);
    const int o = r == 13 ? F : g.cmap[F * 64 + (cz * 4 + cy) * 4 + cx];
    const bool same = r == 13 || g.poff[(int64_t)F * 27 + r] < 0;
    const uint64_t t = same ? g.stab[(int64_t)o * 8 + w] : 0ull;
    tab[r][2 * w] = uint32_t(t);
    tab[r][2 * w + 1] = uint32_t(t >> 32);
  }
  if (tid < 96) {
    const int a = tid >> 5, c = tid & 31;
    const SubstAxis& s = a == 0 ? ax : (a == 1 ? ay : az);
    if (c < s.nL) {
      const int v = c < s.nE ? s.e0 + 2 * c : s.o0 + 2 * (c - s.nE);
      const int rg = v < 0 ? 0 : (v < NB ? 1 : 2);
      const int l = v - (rg - 1) * NB;
      const int bits = (int(l < FL) << a) | (int(l >= BL) << (3 + a)) | ((v & 1) << (6 + a));
      lut[a][c] = make_int2(v, rg * (a == 0 ? 1 : (a == 1 ? 3 : 9)) + (bits << 8));
    }
  }
  const int L0 = ax.nL, L1 = ay.nL;
  const int L01 = L0 * L1;
  const int nV = L01 * az.nL;
  // LDS: the lattice values, their slab flags as a bit mask (64 lattice
  // points a word), then the temporaries of the tensor sums
  T* V = reinterpret_cast<T*>(lds_raw);
  const int vbytes = (nV * int(sizeof(T)) + 7) & ~7;
  uint64_t* FLW = reinterpret_cast<uint64_t*>(lds_raw + vbytes);
  const uint32_t* FL32 = reinterpret_cast<const uint32_t*>(FLW);
  T* TMP = reinterpret_cast<T*>(lds_raw + vbytes + ((nV + 63) >> 6) * 8);
  auto flag = [&](int p) { return (FL32[p >> 5] >> (p & 31)) & 1u; };
  __syncthreads();
  {
    // stage the lattice, value and slab flag; U loads in flight per thread
    // (lanes past the lattice's end work on its point 0 and store nothing)
    constexpr int U = 8;
    const T* fld = g.field;
    Iter3 q(tid, nt, L0, L1);
    for (int i0 = tid; i0 < nV; i0 += U * nt) {
      T v[U];
      uint32_t fl[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        fl[u] = 0u;
        if (i0 + u * nt < nV) {
          const int2 ex = lut[0][q.x], ey = lut[1][q.y], ez = lut[2][q.z];
          const int sum = ex.y + ey.y + ez.y;
          const int r = sum & 31, bits = sum >> 8;
          const SDesc d = desc[r];
          const int e = ex.x + __mul24(ey.x, d.sy) + __mul24(ez.x, d.sz);
          v[u] = fld[d.off + e];
          fl[u] = (tab[r][bits >> 5] >> (bits & 31)) & 1u;
        }
        q.advance();
      }
      // the 64 lanes of a wave hold 64 consecutive lattice points from a
      // multiple of 64 on; lane 0, the wave's first, writes their flag word
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * nt;
        const uint64_t m = __ballot(i < nV && fl[u] != 0u);
        if (i < nV) {
          V[i] = v[u];
          if ((tid & 63) == 0) FLW[i >> 6] = m;
        }
      }
    }
  }
  __syncthreads();
  // degree 1: odd along one axis, the N even neighbours along it
  for_box(ax.nO, ay.nE, az.nE, [&](int i, int j, int k) {
    const int row = imad24(imad24(k, L1, j), L0, 0);
    const int p = row + ax.nE + i;
    if (flag(p)) V[p] = -gtaps<T, N>(V + row + i, 1);
  });
  for_box(ax.nE, ay.nO, az.nE, [&](int i, int j, int k) {
    const int p = imad24(imad24(k, L1, ay.nE + j), L0, i);
    if (flag(p)) V[p] = -gtaps<T, N>(V + imad24(imad24(k, L1, j), L0, i), L0);
  });
  for_box(ax.nE, ay.nE, az.nO, [&](int i, int j, int k) {
    const int p = imad24(imad24(az.nE + k, L1, j), L0, i);
    if (flag(p)) V[p] = -gtaps<T, N>(V + imad24(imad24(k, L1, j), L0, i), L01);
  });
  __syncthreads();
  // degree 2: the tensor sum along the second odd axis into a temporary,
  // without the central term where that would be the point itself, then
  // along the first odd axis (the temporary's odd entry holds the other taps
  // of the point's own column).  The (x, y) and (x, z) classes share one
  // round and the (y, z) class reuses their temporaries' space; a degree-2
  // point reads only points of degree 0 and 1, so the order of the classes
  // does not matter.
  {
    T* Txy = TMP;                                 // [nE_z][nO_y][L0]
    T* Txz = Txy + az.nE * ay.nO * L0;            // [nO_z][nE_y][L0]
    for_box(L0, ay.nO, az.nE, [&](int c, int j, int k) {
      T v = gtaps<T, N>(V + imad24(imad24(k, L1, j), L0, c), L0);
      if (c < ax.nE) v += V[imad24(imad24(k, L1, ay.nE + j), L0, c)];
      Txy[imad24(imad24(k, ay.nO, j), L0, c)] = v;
    });
    for_box(L0, ay.nE, az.nO, [&](int c, int j, int k) {
      T v = gtaps<T, N>(V + imad24(imad24(k, L1, j), L0, c), L01);
      if (c < ax.nE) v += V[imad24(imad24(az.nE + k, L1, j), L0, c)];
      Txz[imad24(imad24(k, ay.nE, j), L0, c)] = v;
    });
    __syncthreads();
    for_box(ax.nO, ay.nO, az.nE, [&](int i, int j, int k) {
      const int p = imad24(imad24(k, L1, ay.nE + j), L0, ax.nE + i);
      const T* t = Txy + imad24(imad24(k, ay.nO, j), L0, 0);
      if (flag(p)) V[p] = -(t[ax.nE + i] + gtaps<T, N>(t + i, 1));
    });
    for_box(ax.nO, ay.nE, az.nO, [&](int i, int j, int k) {
      const int p = imad24(imad24(az.nE + k, L1, j), L0, ax.nE + i);
      const T* t = Txz + imad24(imad24(k, ay.nE, j), L0, 0);
      if (flag(p)) V[p] = -(t[ax.nE + i] + gtaps<T, N>(t + i, 1));
    });
    __syncthreads();
  }
  if (az.nO > 0 && ay.nO > 0) {
    T* Tyz = TMP;                                 // [nO_z][L1][nE_x]
    for_box(ax.nE, L1, az.nO, [&](int i, int c, int k) {
      T v = gtaps<T, N>(V + imad24(imad24(k, L1, c), L0, i), L01);
      if (c < ay.nE) v += V[imad24(imad24(az.nE + k, L1, c), L0, i)];
      Tyz[imad24(imad24(k, L1, c), ax.nE, i)] = v;
    });
    __syncthreads();
    for_box(ax.nE, ay.nO, az.nO, [&](int i, int j, int k) {
      const int p = imad24(imad24(az.nE + k, L1, ay.nE + j), L0, i);
      const T* t = Tyz + imad24(imad24(k, L1, 0), ax.nE, i);
      if (flag(p))
        V[p] = -(t[imad24(ay.nE + j, ax.nE, 0)] + gtaps<T, N>(t + imad24(j, ax.nE, 0), ax.nE));
    });
    __syncthreads();
  }
  // degree 3: z, then y, then x; the central term is left out of the z sum
  // at the odd-odd (x, y) columns, which only their own point reads
  if (ax.nO > 0 && ay.nO > 0 && az.nO > 0) {
  T* A = TMP;                                     // [nO_z][L1][L0]
  T* B = A + az.nO * L01;                         // [nO_z][nO_y][L0]
  for_box(L0, L1, az.nO, [&](int cx, int cy, int k) {
    const int a = imad24(imad24(k, L1, cy), L0, cx);
    T v = gtaps<T, N>(V + a, L01);
    if (cx < ax.nE || cy < ay.nE) v += V[imad24(az.nE, L01, a)];
    A[a] = v;
  });
  __syncthreads();
  for_box(L0, ay.nO, az.nO, [&](int c, int j, int k) {
    const T* a = A + imad24(k, L01, c);
    B[imad24(imad24(k, ay.nO, j), L0, c)] =
        a[imad24(ay.nE + j, L0, 0)] + gtaps<T, N>(a + imad24(j, L0, 0), L0);
  });
  __syncthreads();
  for_box(ax.nO, ay.nO, az.nO, [&](int i, int j, int k) {
    const int p = imad24(imad24(az.nE + k, L1, ay.nE + j), L0, ax.nE + i);
    const T* b = B + imad24(imad24(k, ay.nO, j), L0, 0);
    if (flag(p)) V[p] = -(b[ax.nE + i] + gtaps<T, N>(b + i, 1));
  });
  __syncthreads();
  }
  // the box's slab points to the field, in natural order
  T* fb = g.field + (int64_t)F * (NB * NB * NB);
  const int b0 = it.hi[0] - it.lo[0], b1 = it.hi[1] - it.lo[1], b2 = it.hi[2] - it.lo[2];
  for_box(b0, b1, b2, [&](int i, int j, int k) {
    const int x = it.lo[0] + i, y = it.lo[1] + j, z = it.lo[2] + k;
    if (((x | y | z) & 1) == 0) return;
    const int cx = (x & 1) ? ax.nE + ((x - ax.o0) >> 1) : (x - ax.e0) >> 1;
    const int cy = (y & 1) ? ay.nE + ((y - ay.o0) >> 1) : (y - ay.e0) >> 1;
    const int cz = (z & 1) ? az.nE + ((z - az.o0) >> 1) : (z - az.e0) >> 1;
    const int p = imad24(imad24(cz, L1, cy), L0, cx);
    if (flag(p)) fb[(z * NB + y) * NB + x] = V[p];
  });
}

// ------------------------------------------------------ restriction (f->c)
// One workgroup per RItem.  Pass 1 reduces along the item's thinnest axis n:
// each thread reads whole columns of the fine block's ghost-filled field into
// registers and applies H^a at the coarse points of the column.  Passes 2 and
// 3 apply H^a along the two other axes in LDS.
template <typename T, int N, int NT, int NB, int MAXQ>
__global__ __launch_bounds__(256) void k_restrict(DevGrid<T> g, const RItem* __restrict__ items) {
  extern __shared__ unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  __shared__ Desc desc[27];
  __shared__ CellTab ct;
  constexpr int H = Ha<N, NT>::R;
  constexpr int XS = 2 * (MAXQ - 1) + 1 + 2 * H;
  const RItem it = items[xcd_item(blockIdx.x, gridDim.x)];
  const int F = it.fblk;
  const int tid = threadIdx.x;
  const int L = g.lev[F];
  if (tid < 27) {
    make_desc(g, F, tid, desc[tid]);
    if (tid != 13) {
      const int rx = tid % 3, ry = (tid / 3) % 3, rz = tid / 9;
      const int cx = rx == 0 ? 0 : (rx == 1 ? 1 : 3);
      const int cy = ry == 0 ? 0 : (ry == 1 ? 1 : 3);
      const int cz = rz == 0 ? 0 : (rz == 1 ? 1 : 3);
      if (g.lev[g.cmap[F * 64 + (cz * 4 + cy) * 4 + cx]] > L) desc[tid].patch = 2;  // injection
    }
  }
  load_cells(g, F, ct);
  int qlo[3], qs[3], xlo[3], xs[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    qlo[a] = it.lo[a] - it.sh[a];
    qs[a] = it.hi[a] - it.lo[a];
    xlo[a] = 2 * qlo[a] - H;
    xs[a] = 2 * (qs[a] - 1) + 1 + 2 * H;
  }
  // reduction order: n (thinnest), then a1, then a2
  // pass 1 runs along y or z (the thinner of the two), so that the lanes of
  // a wave, which walk along x, read consecutive addresses
  const int n = qs[1] <= qs[2] ? 1 : 2;
  const int a1 = 0, a2 = n == 2 ? 1 : 2;
  T* R1 = lds;                               // [xs_a2][xs_a1][qs_n]
  T* R2 = R1 + qs[n] * xs[a1] * xs[a2];      // [xs_a2][qs_a1][qs_n]
  const int ox = g.ijk[3 * F] * NB, oy = g.ijk[3 * F + 1] * NB, oz = g.ijk[3 * F + 2] * NB;
  const int nt = blockDim.x;
  __syncthreads();
  {
    const int ncol = xs[a1] * xs[a2];
    // unit step along n and column origin, as scalars (no runtime-indexed
    // arrays, which would live in scratch memory)
    const int ex = n == 0, ey = n == 1, ez = n == 2;
    for (int cidx = tid; cidx < ncol; cidx += nt) {
      const int c1 = cidx % xs[a1], c2 = cidx / xs[a1];
      const int b1 = xlo[a1] + c1, b2 = xlo[a2] + c2;
      const int px0 = n == 0 ? xlo[0] : (a1 == 0 ? b1 : b2);
      const int py0 = n == 1 ? xlo[1] : (a1 == 1 ? b1 : b2);
      const int pz0 = n == 2 ? xlo[2] : (a1 == 2 ? b1 : b2);
      // The column crosses at most three regions along n (before, inside,
      // after the block); the two other coordinates are fixed, so each
      // region is a pointer and a stride.  Every load of the column is
      // issued before the first use; positions past the column end are
      // clamped onto its last point (never used).
      const int pn0 = n == 0 ? px0 : (n == 1 ? py0 : pz0);
      const T* sp[3];
      int32_t sst[3];
      bool inj = false;
#pragma unroll
      for (int rn = 0; rn < 3; ++rn) {
        const int qx = n == 0 ? (rn == 0 ? -1 : (rn == 1 ? 0 : NB)) : px0;
        const int qy = n == 1 ? (rn == 0 ? -1 : (rn == 1 ? 0 : NB)) : py0;
        const int qz = n == 2 ? (rn == 0 ? -1 : (rn == 1 ? 0 : NB)) : pz0;
        const int rx = qx < 0 ? 0 : (qx < NB ? 1 : 2);
        const int ry = qy < 0 ? 0 : (qy < NB ? 1 : 2);
        const int rz = qz < 0 ? 0 : (qz < NB ? 1 : 2);
        const Desc d = desc[rx + 3 * ry + 9 * rz];
        const int32_t st = n == 0 ? 1 : (n == 1 ? d.sy : d.sz);
        // pointer of the column's position 0 (coordinate pn0) in this region
        const int bx = n == 0 ? pn0 : px0, by = n == 1 ? pn0 : py0, bz = n == 2 ? pn0 : pz0;
        sp[rn] = (d.patch == 1 ? g.patch : g.field) + d.off + bx + (int64_t)by * d.sy +
                 (int64_t)bz * d.sz;
        sst[rn] = st;
        const bool used = rn == 0 ? pn0 < 0 : (rn == 1 ? (pn0 < NB && pn0 + xs[n] > 0)
                                                        : pn0 + xs[n] > NB);
        inj = inj || (used && d.patch == 2);
      }
      // region boundaries along the column: the column start is the item's
      // xlo[n] for every lane, so the segment of each load is uniform
      const int xs_n = __builtin_amdgcn_readfirstlane(xs[n]);
      const int j0 = __builtin_amdgcn_readfirstlane(-xlo[n]);
      const int j1 = __builtin_amdgcn_readfirstlane(NB - xlo[n]);
      T col[XS];
      if (!inj) {
#pragma unroll
        for (int j = 0; j < XS; ++j) {
          const int jj = j < xs_n ? j : xs_n - 1;
          if (jj < j0) col[j] = sp[0][jj * sst[0]];
          else if (jj < j1) col[j] = sp[1][jj * sst[1]];
          else col[j] = sp[2][jj * sst[2]];
        }
      } else {
        // a finer-still leaf inside the window: resolve every point
        int bad = 0;
#pragma unroll
        for (int j = 0; j < XS; ++j) {
          const int jj = j < xs[n] ? j : xs[n] - 1;
          const int px = px0 + ex * jj, py = py0 + ey * jj, pz = pz0 + ez * jj;
          const int rx = px < 0 ? 0 : (px < NB ? 1 : 2);
          const int ry = py < 0 ? 0 : (py < NB ? 1 : 2);
          const int rz = pz < 0 ? 0 : (pz < NB ? 1 : 2);
          const Desc d = desc[rx + 3 * ry + 9 * rz];
          int64_t e = d.off + px + (int64_t)py * d.sy + (int64_t)pz * d.sz;
          if (d.patch == 2) e = cell_index<NB>(ct, L, ox, oy, oz, px, py, pz, bad);
          col[j] = (d.patch == 1 ? g.patch : g.field)[e];
        }
        if (bad) atomicAdd(g.err, 1);
      }
      T* dst = R1 + cidx * qs[n];
#pragma unroll
      for (int k = 0; k < MAXQ; ++k) {
        if (k < qs[n]) {
          T acc = T(0);
#pragma unroll
          for (int o = -H; o <= H; ++o)
            if (Ha<N, NT>::c(o) != 0.0) acc += T(Ha<N, NT>::c(o)) * col[2 * k + H + o];
          dst[k] = acc;
        }
      }
    }
  }
  __syncthreads();
  {
    const int cnt = qs[n] * qs[a1] * xs[a2];
    Iter3 q(tid, nt, qs[n], qs[a1]);
    for (int i = tid; i < cnt; i += nt, q.advance()) {
      const T* src = R1 + (q.z * xs[a1] + 2 * q.y + H) * qs[n] + q.x;
      T acc = T(0);
#pragma unroll
      for (int o = -H; o <= H; ++o)
        if (Ha<N, NT>::c(o) != 0.0) acc += T(Ha<N, NT>::c(o)) * src[o * qs[n]];
      R2[i] = acc;
    }
  }
  __syncthreads();
  {
    const int cnt = qs[n] * qs[a1] * qs[a2];
    Iter3 q(tid, nt, qs[n], qs[a1]);
    for (int i = tid; i < cnt; i += nt, q.advance()) {
      const T* src = R2 + ((2 * q.z + H) * qs[a1] + q.y) * qs[n] + q.x;
      T acc = T(0);
#pragma unroll
      for (int o = -H; o <= H; ++o)
        if (Ha<N, NT>::c(o) != 0.0) acc += T(Ha<N, NT>::c(o)) * src[o * qs[a1] * qs[n]];
      const int c0 = n == 0 ? q.x : (a1 == 0 ? q.y : q.z);
      const int cy1 = n == 1 ? q.x : (a1 == 1 ? q.y : q.z);
      const int cz2 = n == 2 ? q.x : (a1 == 2 ? q.y : q.z);
      g.patch[it.off + ((int64_t)(it.lo[2] + cz2 - it.rlo[2]) * it.rsz[1] + (it.lo[1] + cy1 - it.rlo[1])) * it.rsz[0] +
              (it.lo[0] + c0 - it.rlo[0])] = acc;
    }
  }
}

template <int FD> struct FDW;
// central schemes: d/dx ~ sum_k c(k) (f[+k] - f[-k]) / h and, for the
// diffusion operator (DIFF-2 / DIFF-4 of the finite-difference supplement,
// and order 6), d2/dx2 ~ (d2(0) f[0] + sum_k d2(k) (f[+k] + f[-k])) / h^2
template <> struct FDW<2> {
  static constexpr int G = 1;
  static constexpr bool CONS = false;
  __device__ static constexpr double c(int) { return 0.5; }
  __device__ static constexpr double d2(int k) { return k == 0 ? -2.0 : 1.0; }
  __device__ static constexpr double cp(int) { return 0.0; }
  __device__ static constexpr double cm(int) { return 0.0; }
};
template <> struct FDW<4> {
  static constexpr int G = 2;
  static constexpr bool CONS = false;
  __device__ static constexpr double c(int k) { return k == 1 ? 8.0 / 12.0 : -1.0 / 12.0; }
  __device__ static constexpr double d2(int k) {
    return k == 0 ? -30.0 / 12.0 : (k == 1 ? 16.0 / 12.0 : -1.0 / 12.0);
  }
  __device__ static constexpr double cp(int) { return 0.0; }
  __device__ static constexpr double cm(int) { return 0.0; }
};
template <> struct FDW<6> {
  static constexpr int G = 3;
  static constexpr bool CONS = false;
  __device__ static constexpr double c(int k) {
    return k == 1 ? 45.0 / 60.0 : (k == 2 ? -9.0 / 60.0 : 1.0 / 60.0);
  }
  __device__ static constexpr double d2(int k) {
    return k == 0 ? -490.0 / 180.0
                  : (k == 1 ? 270.0 / 180.0 : (k == 2 ? -27.0 / 180.0 : 2.0 / 180.0));
  }
  __device__ static constexpr double cp(int) { return 0.0; }
  __device__ static constexpr double cm(int) { return 0.0; }
};
// CONS-3 / CONS-5 (finite-difference supplement): the flux difference
// f_{i+1/2} - f_{i-1/2} of the fixed-weight WENO fluxes, sum_r gamma_r S_r of
// the order-3 / order-5 stencil tables, written as one stencil on phi at the
// offsets -G..G: cp for a positive velocity (f^+), cm for a negative one
// (f^-).  With f^+_{i+1/2} = sum_o a_o f_{i+o}, the difference has the weight
// a_o - a_{o+1} at offset o; order 3: a = (-1/6, 5/6, 1/3) at -1..1, order 5:
// a = (2, -13, 47, 27, -3)/60 at -2..2; f^- mirrors them.
template <> struct FDW<3> {
  static constexpr int G = 2;
  static constexpr bool CONS = true;
  __device__ static constexpr double c(int) { return 0.0; }
  __device__ static constexpr double cp(int o) {
    return o == -2 ? 1.0 / 6.0 : o == -1 ? -1.0 : o == 0 ? 0.5 : o == 1 ? 1.0 / 3.0 : 0.0;
  }
  __device__ static constexpr double cm(int o) { return -cp(-o); }
  __device__ static constexpr double d2(int) { return 0.0; }
};
template <> struct FDW<5> {
  static constexpr int G = 3;
  static constexpr bool CONS = true;
  __device__ static constexpr double c(int) { return 0.0; }
  __device__ static constexpr double cp(int o) {
    return o == -3 ? -2.0 / 60.0 : o == -2 ? 15.0 / 60.0 : o == -1 ? -60.0 / 60.0
         : o == 0 ? 20.0 / 60.0 : o == 1 ? 30.0 / 60.0 : o == 2 ? -3.0 / 60.0 : 0.0;
  }
  __device__ static constexpr double cm(int o) { return -cp(-o); }
  __device__ static constexpr double d2(int) { return 0.0; }
};

template <typename T, int FD, int NB>
__global__ __launch_bounds__(NB* NB) void k_rhs(DevGrid<T> g, const T* __restrict__ un,
                                                 T* __restrict__ out, T a_un, T b_y, T c_y, T dt,
                                                 VelDev vel, int first, int nxcd) {
  constexpr int G = FDW<FD>::G;
  constexpr int P = NB + 2 * G;
  constexpr int NH = P * P - NB * NB;
  constexpr int HPT = (NH + NB * NB - 1) / (NB * NB);  // halo points per thread
  __shared__ T plane[P * P];
  __shared__ Desc desc[27];
  __shared__ T vx_z[NB], vy_x[NB], vz_y[NB];
  // XCD-aware order: consecutive workgroups are dispatched round-robin to the
  // XCDs, so give each XCD one contiguous run of (Morton-ordered) blocks.
  // Workgroup i runs on XCD x = i % nxcd as its k = i / nxcd-th; XCD x owns
  // blocks [x*q + min(x, r), ...) with q = n / nxcd, r = n % nxcd (bijection).
  const int nblk = gridDim.x;
  const int q = nblk / nxcd, rem = nblk % nxcd;
  const int xcd = blockIdx.x % nxcd, kk0 = blockIdx.x / nxcd;
  const int bl = xcd * q + (xcd < rem ? xcd : rem) + kk0;
  const int b = first + bl;
  const int tid = threadIdx.x;
  if (tid < 27) make_desc(g, b, tid, desc[tid]);
  const int nb = NB;
  const int L = g.lev[b];
  const double den = double(nb << L);
  const double inv_h = den;
  if (tid < NB) {
    const double xi = (double(g.ijk[3 * b] * nb + tid)) / den;
    const double yi = (double(g.ijk[3 * b + 1] * nb + tid)) / den;
    const double zi = (double(g.ijk[3 * b + 2] * nb + tid)) / den;
    if (vel.kind == 2) {
      const double tp = 6.283185307179586;
      vx_z[tid] = T(sin(tp * zi));
      vy_x[tid] = T(sin(tp * xi));
      vz_y[tid] = T(sin(tp * yi));
    } else if (vel.kind == 1) {
      vx_z[tid] = T(-(yi - vel.p[1]));  // u_x depends on y
      vy_x[tid] = T(xi - vel.p[0]);     // u_y depends on x
      vz_y[tid] = T(vel.p[2]);
    } else {
      vx_z[tid] = T(vel.p[0]);
      vy_x[tid] = T(vel.p[1]);
      vz_y[tid] = T(vel.p[2]);
    }
  }
  __syncthreads();
  const int tx = tid % NB, ty = tid / NB;
  const T* fbuf = g.field;
  const T* pbuf = g.patch;
  auto load = [&](int x, int y, int z) -> T {
    const int rx = x < 0 ? 0 : (x < NB ? 1 : 2);
    const int ry = y < 0 ? 0 : (y < NB ? 1 : 2);
    const int rz = z < 0 ? 0 : (z < NB ? 1 : 2);
    const Desc d = desc[rx + 3 * ry + 9 * rz];
    const T* buf = d.patch ? pbuf : fbuf;
    return buf[d.off + x + (int64_t)y * d.sy + (int64_t)z * d.sz];
  };
  // halo points of this thread: t = tid + k*NB*NB.  Enumeration of the ring:
  // rows y in [-G,0) and [NB,NB+G) fully, then the side columns of rows [0,NB)
  int hx[HPT], hy[HPT];
  bool hh[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    int t = tid + k * NB * NB;
    hh[k] = t < NH;
    hx[k] = 0;
    hy[k] = 0;
    if (hh[k]) {
      const int full = G * P;
      if (t < 2 * full) {
        const int row = t / P, c = t % P;
        hy[k] = row < G ? row - G : NB + (row - G);
        hx[k] = c - G;
      } else {
        t -= 2 * full;
        const int row = t / (2 * G), c = t % (2 * G);
        hy[k] = row;
        hx[k] = c < G ? c - G : NB + (c - G);
      }
    }
  }
  // Loads run two planes ahead of the stencil: col holds planes z-G..z+G,
  // pf1 plane z+G+1 and the halo values of plane z+1 (hv1); at plane z the
  // loads of plane z+G+2 and of the halo of z+2 are issued.
  T col[2 * G + 1];
#pragma unroll
  for (int i = 0; i < 2 * G + 1; ++i) col[i] = load(tx, ty, i - G);
  T pf1 = load(tx, ty, G + 1);
  // threads without a halo point load their own interior point instead, so
  // that every thread issues the same number of loads per plane (partial
  // vmcnt waits instead of full drains)
#pragma unroll
  for (int k = 0; k < HPT; ++k)
    if (!hh[k]) {
      hx[k] = tx;
      hy[k] = ty;
    }
  T hval[HPT], hv1[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    hval[k] = load(hx[k], hy[k], 0);
    hv1[k] = load(hx[k], hy[k], 1);
  }
  const int64_t nb3 = (int64_t)NB * NB * NB;
  const int64_t obase = (int64_t)b * nb3 + (int64_t)ty * NB + tx;
  const T ux_y = vx_z[ty];  // rotating: u_x = -(y - cy) (per y); shear: per z
  // u^n is also read one plane ahead, before that plane's stencil loads, so
  // waiting for it never drains the loads issued later.  u^n and the output
  // are touched once per point: non-temporal accesses leave more of L2 to
  // the stage input, whose rows are read again as the neighbours' halos.
  T ucur = __builtin_nontemporal_load(&un[obase]);
  // fully unrolled: the register rotations below become renames, so the
  // loads issued for later planes stay in flight across iterations
#pragma unroll
  for (int z = 0; z < NB; ++z) {
    plane[(ty + G) * P + tx + G] = col[G];
#pragma unroll
    for (int k = 0; k < HPT; ++k)
      if (hh[k]) plane[(hy[k] + G) * P + hx[k] + G] = hval[k];
    const T u0 = ucur;
    if (z + 1 < NB) ucur = __builtin_nontemporal_load(&un[obase + (int64_t)(z + 1) * NB * NB]);
    T pf2 = T(0), hv2[HPT];
    if (z + G + 2 < NB + G) pf2 = load(tx, ty, z + G + 2);
#pragma unroll
    for (int k = 0; k < HPT; ++k) hv2[k] = (z + 2 < NB) ? load(hx[k], hy[k], z + 2) : T(0);
    __syncthreads();
    T dx = T(0), dy = T(0), dz = T(0);
    T dxm = T(0), dym = T(0), dzm = T(0);
    if (!FDW<FD>::CONS && vel.kind == 3) {
      // diffusion: nu times the sum of the three second differences
      const int c0 = (ty + G) * P + tx + G;
      T lap = T(3.0 * FDW<FD>::d2(0)) * col[G];
#pragma unroll
      for (int kk = 1; kk <= G; ++kk)
        lap += T(FDW<FD>::d2(kk)) * ((plane[c0 + kk] + plane[c0 - kk]) +
                                     (plane[c0 + kk * P] + plane[c0 - kk * P]) +
                                     (col[G + kk] + col[G - kk]));
      dx = T(-vel.p[0] * inv_h) * lap;   // rhs = -(dx) * inv_h below
    } else if constexpr (!FDW<FD>::CONS) {
#pragma unroll
      for (int kk = 1; kk <= G; ++kk) {
        const T c = T(FDW<FD>::c(kk));
        dx += c * (plane[(ty + G) * P + tx + G + kk] - plane[(ty + G) * P + tx + G - kk]);
        dy += c * (plane[(ty + G + kk) * P + tx + G] - plane[(ty + G - kk) * P + tx + G]);
        dz += c * (col[G + kk] - col[G - kk]);
      }
    } else {
      // both upwind differences; the sign of each velocity component picks
      // one below
#pragma unroll
      for (int o = -G; o <= G; ++o) {
        const T cp = T(FDW<FD>::cp(o)), cm = T(FDW<FD>::cm(o));
        const T fx = plane[(ty + G) * P + tx + G + o];
        const T fy = plane[(ty + G + o) * P + tx + G];
        const T fz = col[G + o];
        if (FDW<FD>::cp(o) != 0.0) {
          dx += cp * fx;
          dy += cp * fy;
          dz += cp * fz;
        }
        if (FDW<FD>::cm(o) != 0.0) {
          dxm += cm * fx;
          dym += cm * fy;
          dzm += cm * fz;
        }
      }
    }
    T ux, uy, uz;
    if (vel.kind == 3) {
      ux = T(1);
      uy = uz = T(0);
    } else if (vel.kind == 2) {
      ux = vx_z[z];
      uy = vy_x[tx];
      uz = vz_y[ty];
    } else if (vel.kind == 1) {
      ux = ux_y;
      uy = vy_x[tx];
      uz = vz_y[0];
    } else {
      ux = vx_z[0];
      uy = vy_x[0];
      uz = vz_y[0];
    }
    if constexpr (FDW<FD>::CONS) {
      // u_d does not vary along x_d for these velocity fields, so the
      // interface velocity u_{i+1/2} is u_d at the point
      dx = ux > T(0) ? dx : dxm;
      dy = uy > T(0) ? dy : dym;
      dz = uz > T(0) ? dz : dzm;
    }
    const T rhs = -(ux * dx + uy * dy + uz * dz) * T(inv_h);
    const T yv = col[G];
    const T res = c_y == T(1) ? a_un * u0 + b_y * (yv + dt * rhs)
                              : a_un * u0 + b_y * (c_y * yv + dt * rhs);
    __builtin_nontemporal_store(res, &out[obase + (int64_t)z * NB * NB]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2 * G; ++i) col[i] = col[i + 1];
    col[2 * G] = pf1;
    pf1 = pf2;
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      hval[k] = hv1[k];
      hv1[k] = hv2[k];
    }
  }
}

// smallest v' >= v with v' = rem (mod m)
constexpr int pad_to(int v, int m, int rem) { return v + ((rem - v % m) % m + m) % m; }

// Lifting form of the analysis pair: G^a at an odd point is the point minus
// the DD prediction from the N even points around it; for Nt = 2, H^a at an
// even point is the point plus a quarter of the two G^a values beside it
// (the update that gives H^a its taps).  w is a window of values, i the odd
// point's index in it.
template <int N>
__device__ __forceinline__ double lift_gamma(const double* w, int i) {
  double g = w[i];
#pragma unroll
  for (int k = 0; k < N; ++k) g -= DD<N>::w(k) * w[i - 1 + 2 * (k + DD<N>::J0)];
  return g;
}

// Smallest stride s >= nb (in 8-byte words) with step * s = nb (mod 16), or
// nb when there is none below nb + 16.
constexpr int y_row_stride(int nb, int step) {
  for (int s = nb; s < nb + 16; ++s)
    if ((step * s - nb) % 16 == 0) return s;
  return nb;
}

// Smallest row stride >= v (in 4-byte words) for which 32 lanes reading
// word r * stride + step * t (lane = r * per_row + t, t < per_row) hit 32
// distinct LDS banks; v itself when no stride below v + 32 does.
constexpr int bank_free_stride(int v, int per_row, int step) {
  for (int s = v; s < v + 32; ++s) {
    unsigned used = 0;
    bool ok = true;
    for (int l = 0; l < 32 && ok; ++l) {
      const int b = ((l / per_row) * s + step * (l % per_row)) % 32;
      ok = !((used >> b) & 1u);
      used |= 1u << b;
    }
    if (ok) return s;
  }
  return v;
}
// ------------------------------------------------------------------ details
// Forward transform (x, then y, then z) of the ghost-filled block in FP64,
// per-block maxima of |gamma| over 27 (x-class, y-class, z-class) boxes:
// class 0 = [0, nb), 1 = [0, eb), 2 = [nb-ef, nb).
// Planes are taken ZG at a time: every barrier phase (staging, x pass,
// y pass) works on the whole group, so a plane costs 3/ZG barriers.  The
// input planes are staged in the field's precision (exact) and converted
// when read; the x pass computes XP consecutive (H^a, G^a) pairs of a row
// per thread and the y pass YP pairs of a column, so that a value read from
// LDS serves several outputs.  Every pass uses the lifting form of the
// filters (lift_gamma), half the multiply-adds of the H^a / G^a taps.  With
// 24^3 blocks one workgroup fills a CU whatever its LDS (registers limit
// it), so the group is 4 planes; smaller blocks keep it at 2 so that LDS
// does not cap the workgroups per CU.
template <typename T, int NB, int N, int NT, int ZG = (NB >= 24 ? 4 : 2), int PF = 4>
__global__ __launch_bounds__(NB* NB) void k_details(DevGrid<T> g, int ef, int eb,
                                                     double* __restrict__ bands,
                                                     const int32_t* __restrict__ det_slot,
                                                     double* __restrict__ det_out, int first) {
  constexpr int HR = Ha<N, NT>::R;
  constexpr int GR = Ga<N>::R;
  constexpr int HF = HR > GR - 1 ? HR : GR - 1;        // front ghost depth
  constexpr int HB = (HR - 1) > GR ? (HR - 1) : GR;    // back ghost depth
  constexpr int R = HR > GR ? HR : GR;                 // z ring half-width
  constexpr int P = NB + HF + HB;
  constexpr int LPT = (P * P + NB * NB - 1) / (NB * NB);
  constexpr int NP = NB / 2;
  constexpr int XP = NP % 3 == 0 ? 3 : (NP % 2 == 0 ? 2 : 1);   // pairs per x task
  constexpr int YP = NP % 2 == 0 ? 2 : 1;                       // pairs per y task
  constexpr int XT = NP / XP, YT = NP / YP;                    // tasks per row, column
  // offsets (from the first pair's even point) of the values a task reads
  constexpr int DLO = -(HR > GR - 1 ? HR : GR - 1);
  constexpr int DHX = 2 * (XP - 1) + (HR > GR + 1 ? HR : GR + 1);
  constexpr int DHY = 2 * (YP - 1) + (HR > GR + 1 ? HR : GR + 1);
  static_assert(PF >= ZG, "a group's planes are loaded before it starts");
  // LDS layout, chosen so that the lanes of one access fall on distinct
  // banks (32 banks of 4 bytes):
  // * a staged plane is split into its even and odd x columns (x counted
  //   from the block origin), so the x pass reads consecutive values; the
  //   row stride PH puts the 32 lanes of a half-wave (rows of XT tasks,
  //   XP values apart) on distinct banks (4-byte values), or continues the
  //   banks of the previous row (8-byte values, PH = NP mod 16); the odd
  //   half starts 16 banks after the even half;
  // * x-pass rows of NBS doubles for the y pass, whose lanes take a row's NB
  //   columns and then the same columns 2 YP rows further: 2 YP NBS = NB
  //   (mod 16) makes the second row continue the first one's banks.
  constexpr int PH = sizeof(T) == 4 ? bank_free_stride((P + 1) / 2, XT, XP)
                                    : pad_to((P + 1) / 2, 16, NP % 16);
  constexpr int PS = sizeof(T) == 4 ? pad_to(P * PH, 32, 16) : pad_to(P * PH, 16, 8);
  constexpr int NBS = y_row_stride(NB, 2 * YP);
  __shared__ __align__(16) T pl[ZG][2 * PS];   // input planes: even, odd columns
  __shared__ double t1[ZG][P * NBS];  // after the x pass
  __shared__ double t2[ZG][NB * NB];  // after the y pass
  __shared__ Desc desc[27];
  __shared__ int nonfinite;
  // XCD-aware order: a block's halo is its Morton neighbours' data, which
  // then sits in the same XCD's L2
  const int b = first + xcd_item(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int slot = __builtin_amdgcn_readfirstlane(det_slot ? det_slot[b] : -1);
  // a pass for the discarded details (det_out given) needs only the blocks
  // with a slot; the others leave at once (the whole workgroup)
  if (det_out && slot < 0) return;
  if (tid < 27) make_desc(g, b, tid, desc[tid]);
  if (tid == 0) nonfinite = 0;
  __syncthreads();
  const int tx = tid % NB, ty = tid / NB;
  const T* fbuf = g.field;
  const T* pbuf = g.patch;
  // Each thread loads the same LPT positions (x, y) of every input plane
  // (clamped onto the last position past the plane's end); their addresses
  // are a pointer plus a z stride per slot, re-based when the fetched plane
  // enters another z region (z < 0, [0, NB), >= NB).
  const T* kp[LPT];
  int32_t ksz[LPT];
  int kx[LPT], ky[LPT], sidx[LPT];
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    int i = tid + k * NB * NB;
    i = i < P * P ? i : P * P - 1;
    kx[k] = i % P - HF;
    ky[k] = i / P - HF;
    const int c = i % P;   // column in the staged plane, x + HF
    sidx[k] = ((c & 1) ^ (HF & 1) ? PS : 0) + (i / P) * PH + (c >> 1);
  }
  auto rebase = [&](int rz) {
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int rx = kx[k] < 0 ? 0 : (kx[k] < NB ? 1 : 2);
      const int ry = ky[k] < 0 ? 0 : (ky[k] < NB ? 1 : 2);
      const Desc d = desc[rx + 3 * ry + 9 * rz];
      kp[k] = (d.patch ? pbuf : fbuf) + d.off + kx[k] + (int64_t)ky[k] * d.sy;
      ksz[k] = d.sz;
    }
  };
  auto fetch = [&](T* dst, int z) {
#pragma unroll
    for (int k = 0; k < LPT; ++k) dst[k] = kp[k][(int64_t)z * ksz[k]];
  };
  auto zreg = [](int z) { return z < 0 ? 0 : (z < NB ? 1 : 2); };
  double ring[2 * R + 1];
#pragma unroll
  for (int i = 0; i < 2 * R + 1; ++i) ring[i] = 0.0;   // planes below -HF: no tap reaches them
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  double gz = 0.0;   // G^a of the last odd plane computed ahead (Nt = 2)
  bool bad = false;
  // PF planes in flight (a register ring); the whole plane loop is unrolled,
  // so plane index, region changes, output parity and the ring rotations
  // are resolved at compile time
  constexpr int ZLAST = NB + HB - 1;   // last input plane
  T nx[PF][LPT];
#pragma unroll
  for (int q = 0; q < PF; ++q) {
    const int z = -HF + q;
    if (z <= ZLAST) {
      if (q == 0 || zreg(z) != zreg(z - 1)) rebase(zreg(z));
      fetch(nx[q], z);
    }
  }
#pragma unroll
  for (int z0 = -HF; z0 < NB + R; z0 += ZG) {
    const bool live = z0 <= ZLAST;   // the group holds an input plane
    // stage the group's planes in LDS, then reuse their load slots for the
    // planes PF ahead (issued in z order: each re-base follows the last)
#pragma unroll
    for (int q = 0; q < ZG; ++q) {
      const int zi = z0 + q;
      if (zi <= ZLAST) {
        const T* cur = nx[(zi + HF) % PF];
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
          const int i = tid + k * NB * NB;
          if (k < LPT - 1 || i < P * P) pl[q][sidx[k]] = cur[k];
        }
      }
    }
    if (live) __syncthreads();
#pragma unroll
    for (int q = 0; q < ZG; ++q) {
      const int zi = z0 + q;
      if (zi <= ZLAST && zi + PF <= ZLAST) {
        if (zreg(zi + PF) != zreg(zi + PF - 1)) rebase(zreg(zi + PF));
        fetch(nx[(zi + HF) % PF], zi + PF);
      }
    }
    if (live) {
      // x pass: H^a at the even points 2j, G^a at 2j+1 of each row, for XP
      // consecutive pairs j0 .. j0+XP-1 per thread, every plane of the group
      for (int i = tid; i < ZG * P * XT; i += NB * NB) {
        const int jt = i % XT, rq = i / XT;
        const int q = rq / P, yy = rq % P;
        if (z0 + q > ZLAST) continue;
        const int j0 = jt * XP;
        // the value at x = 2 j0 + d: even or odd half by the parity of d
        const T* row = pl[q] + yy * PH + j0;
        double w[DHX - DLO + 1];
#pragma unroll
        for (int d = DLO; d <= DHX; ++d)
          w[d - DLO] = double((d & 1) ? row[PS + ((d + HF) >> 1)] : row[(d + HF) >> 1]);
        double gm[XP + 1];   // G^a at the odd points 2p - 1, p = 0 .. XP
#pragma unroll
        for (int p = NT ? 0 : 1; p <= XP; ++p) gm[p] = lift_gamma<N>(w, 2 * p - 1 - DLO);
#pragma unroll
        for (int p = 0; p < XP; ++p) {
          const double ev = NT ? w[2 * p - DLO] + 0.25 * (gm[p] + gm[p + 1]) : w[2 * p - DLO];
          t1[q][yy * NBS + 2 * (j0 + p)] = ev;
          t1[q][yy * NBS + 2 * (j0 + p) + 1] = gm[p + 1];
        }
      }
      __syncthreads();
      // y pass: (plane, column x, rows 2j (H^a) and 2j+1 (G^a)) for YP
      // consecutive pairs per thread
      for (int i = tid; i < ZG * NB * YT; i += NB * NB) {
        const int x = i % NB, r = i / NB;
        const int jt = r % YT, q = r / YT;
        if (z0 + q > ZLAST) continue;
        const int j0 = jt * YP;
        const double* col = t1[q] + (2 * j0 + HF) * NBS + x;
        double w[DHY - DLO + 1];
#pragma unroll
        for (int d = DLO; d <= DHY; ++d) w[d - DLO] = col[d * NBS];
        double gm[YP + 1];
#pragma unroll
        for (int p = NT ? 0 : 1; p <= YP; ++p) gm[p] = lift_gamma<N>(w, 2 * p - 1 - DLO);
#pragma unroll
        for (int p = 0; p < YP; ++p) {
          const double ev = NT ? w[2 * p - DLO] + 0.25 * (gm[p] + gm[p + 1]) : w[2 * p - DLO];
          t2[q][2 * (j0 + p) * NB + x] = ev;
          t2[q][(2 * (j0 + p) + 1) * NB + x] = gm[p + 1];
        }
      }
      __syncthreads();
    }
    // z pass over the group's planes, in order, through the register ring
#pragma unroll
    for (int q = 0; q < ZG; ++q) {
      const int zi = z0 + q;
      const double v = zi <= ZLAST ? t2[q][ty * NB + tx] : 0.0;
#pragma unroll
      for (int i = 0; i < 2 * R; ++i) ring[i] = ring[i + 1];
      ring[2 * R] = v;
      const int zo = zi - R;
      if (zo >= 0 && zo < NB) {
        // ring[R + o] holds plane zo + o; with Nt = 2 the G^a value of the
        // odd plane after an even output is computed with it and kept for
        // that plane's own output (gz), as is the one before (gz, or the
        // plane -1's at zo = 0)
        double gsum;
        if ((zo & 1) == 0) {
          if (NT) {
            const double gp = zo == 0 ? lift_gamma<N>(ring, R - 1) : gz;
            gz = lift_gamma<N>(ring, R + 1);
            gsum = ring[R] + 0.25 * (gp + gz);
          } else {
            gsum = ring[R];
          }
        } else {
          gsum = NT ? gz : lift_gamma<N>(ring, R);
        }
        const bool isdet = (zo & 1) != 0 || ((tx | ty) & 1) != 0;
        const double a = isdet ? fabs(gsum) : 0.0;
        bad = bad || !(a <= 1e300);
        m0 = fmax(m0, a);
        if (zo < eb) m1 = fmax(m1, a);
        if (zo >= NB - ef) m2 = fmax(m2, a);
        if (slot >= 0)
          det_out[(int64_t)slot * NB * NB * NB + ((int64_t)zo * NB + ty) * NB + tx] = isdet ? gsum : 0.0;
      }
    }
  }
  // Fold the column maxima into the 27 boxes (x-class, y-class, z-class;
  // class 0 = [0, nb), 1 = [0, eb), 2 = [nb-ef, nb)) in two LDS stages:
  // per (z-class, row, x-class), then per box over the rows of its y-class.
  // Both folds run over the whole extent with a mask, fully unrolled, so
  // their LDS reads are issued back to back.  (No LDS atomics: a contended
  // atomic max is expanded into a per-lane loop.)  The buffers of the plane
  // loop are free once every thread has passed the first barrier below.
  // (in the x-pass buffer, or the input planes', or a buffer of their own
  // where neither holds them)
  constexpr bool CM_T1 = ZG * P * NBS >= 3 * NB * NB;
  constexpr bool CM_PL = !CM_T1 && ZG * 2 * PS * sizeof(T) >= 3 * NB * NB * sizeof(double);
  __shared__ double cm_own[CM_T1 || CM_PL ? 1 : 3 * NB * NB];
  double* colmax = CM_T1 ? &t1[0][0]
                         : (CM_PL ? reinterpret_cast<double*>(&pl[0][0]) : cm_own);   // [cz][ty][tx]
  double* rowmax = &t2[0][0];          // [cz][ty][cx]
  static_assert(ZG * NB * NB >= 9 * NB, "reduction buffers");
  if (bad) nonfinite = 1;
  __syncthreads();
  colmax[tid] = m0;
  colmax[NB * NB + tid] = m1;
  colmax[2 * NB * NB + tid] = m2;
  __syncthreads();
  for (int i = tid; i < 9 * NB; i += NB * NB) {   // i = (cz * NB + y) * 3 + cx
    const int cx = i % 3, y = (i / 3) % NB, cz = i / (3 * NB);
    const int x0 = cx == 2 ? NB - ef : 0, x1 = cx == 1 ? eb : NB;
    const double* row = colmax + (cz * NB + y) * NB;
    double v = 0.0;
#pragma unroll
    for (int x = 0; x < NB; ++x) {
      const double w = row[x];
      v = (x >= x0 && x < x1) ? fmax(v, w) : v;
    }
    rowmax[i] = v;
  }
  __syncthreads();
  if (tid < 27) {
    const int cx = tid % 3, cy = (tid / 3) % 3, cz = tid / 9;
    const int y0 = cy == 2 ? NB - ef : 0, y1 = cy == 1 ? eb : NB;
    double v = 0.0;
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const double w = rowmax[(cz * NB + y) * 3 + cx];
      v = (y >= y0 && y < y1) ? fmax(v, w) : v;
    }
    if (nonfinite) v = __longlong_as_double(0x7ff8000000000000ll);
    bands[(int64_t)b * 27 + tid] = v;
  }
}

__global__ void k_combine(const int32_t* __restrict__ lev, const int32_t* __restrict__ cmap,
                          const double* __restrict__ bands, int ext, double* __restrict__ norms,
                          int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double v = bands[(int64_t)b * 27 + 0];
  if (ext) {
    const int L = lev[b];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy && !dz) continue;
          const int cx = dx < 0 ? 0 : (dx == 0 ? 1 : 3);
          const int cy = dy < 0 ? 0 : (dy == 0 ? 1 : 3);
          const int cz = dz < 0 ? 0 : (dz == 0 ? 1 : 3);
          const int nbk = cmap[b * 64 + (cz * 4 + cy) * 4 + cx];
          if (lev[nbk] != L) continue;
          // neighbour's boxes next to b: +1 side -> its [0,eb), -1 -> [nb-ef,nb)
          const int kx = dx == 0 ? 0 : (dx > 0 ? 1 : 2);
          const int ky = dy == 0 ? 0 : (dy > 0 ? 1 : 2);
          const int kz = dz == 0 ? 0 : (dz > 0 ? 1 : 2);
          const double w = bands[(int64_t)nbk * 27 + kx + 3 * ky + 9 * kz];
          v = (w > v || w != w) ? w : v;
        }
  }
  norms[b] = v;
}


// ----------------------------------------------------- adaptation passes
// Generic separable pass: one workgroup per PItem, one thread per output
// point.  Scratch boxes are FP64.
template <typename T>
struct PassIO {
  const double* din;
  double* dout;
  const double* det;
  const int32_t* det_slot;
  const uint32_t* det_tab;  // per slot: 16 words, bit (front | back << 3 |
                            // parity << 6) set when the slot's details with
                            // that per-axis slab membership are discarded
  T* dst;  // destination field array (new pool)
};

template <typename T, int N, int NT>
__device__ __forceinline__ double pass_in(const DevGrid<T>& g, const PItem& it, int src_mode,
                                          const PassIO<T>& io, int x, int y, int z) {
  if (src_mode == 0) return double(ext_value(g, it.src_blk, x, y, z));
  if (src_mode == 1) {
    const int ix = x - it.ilo[0], iy = y - it.ilo[1], iz = z - it.ilo[2];
    if ((unsigned)ix >= (unsigned)it.isz[0] || (unsigned)iy >= (unsigned)it.isz[1] ||
        (unsigned)iz >= (unsigned)it.isz[2]) {
      atomicAdd(g.err, 1);
      return 0.0;
    }
    return io.din[it.in_off + ((int64_t)iz * it.isz[1] + iy) * it.isz[0] + ix];
  }
  // src_mode 2: discarded details (old tree): every detail of a coarsening
  // child; of a kept same-level neighbour, every point with an odd index in
  // its coarse-extension slab toward the coarsening children (section 2.2.1,
  // Table 3 coarse region extension: [0, N) in front and [nb-N+1, nb)
  // behind along each facing axis for lifted wavelets, [0, N-1) and
  // [nb-N+2, nb) for N.0), looked up in the slot's table
  const int id = owner_id(g, it.src_blk, 0, x, y, z);
  if (id < 0) return 0.0;
  const int s = io.det_slot[id];
  if (s < 0) return 0.0;
  const int nb = g.nb;
  const int L = g.lev[it.src_blk];
  if (g.lev[id] != L) return 0.0;
  const int W = nb << L;
  // the sample lies within one block of the source block, so one wrap fixes it
  auto wrap1 = [W](int a) { return a < 0 ? a + W : (a >= W ? a - W : a); };
  const int gx = wrap1(g.ijk[3 * it.src_blk] * nb + x) - g.ijk[3 * id] * nb;
  const int gy = wrap1(g.ijk[3 * it.src_blk + 1] * nb + y) - g.ijk[3 * id + 1] * nb;
  const int gz = wrap1(g.ijk[3 * it.src_blk + 2] * nb + z) - g.ijk[3 * id + 2] * nb;
  constexpr int FRONT = NT ? N : N - 1;
  const int back = NT ? nb - N + 1 : nb - N + 2;
  const int bit = int(gx < FRONT) | (int(gy < FRONT) << 1) | (int(gz < FRONT) << 2) |
                  (int(gx >= back) << 3) | (int(gy >= back) << 4) | (int(gz >= back) << 5) |
                  ((gx & 1) << 6) | ((gy & 1) << 7) | ((gz & 1) << 8);
  if (!((io.det_tab[(int64_t)s * 16 + (bit >> 5)] >> (bit & 31)) & 1u)) return 0.0;
  return io.det[(int64_t)s * nb * nb * nb + ((int64_t)gz * nb + gy) * nb + gx];
}

// One instantiation per (filter, source): the unrolled taps of one filter
// and one input path only, so that registers allow several workgroups per
// CU.
template <typename T, int N, int NT, int FILTER, int SRC>
__global__ __launch_bounds__(256) void k_pass(DevGrid<T> g, const PItem* __restrict__ items,
                                              int axis, int dst_mode, PassIO<T> io) {
  constexpr int filter = FILTER, src_mode = SRC;
  const PItem it = items[blockIdx.x];
  int sz[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) sz[a] = it.hi[a] - it.lo[a];
  const int n = sz[0] * sz[1] * sz[2];
  const int nb = g.nb;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  Iter3 qi(threadIdx.x, blockDim.x, sz[0], sz[1]);
  for (int i = threadIdx.x; i < n; i += blockDim.x, qi.advance()) {
    int o[3] = {it.lo[0] + qi.x, it.lo[1] + qi.y, it.lo[2] + qi.z};
    const int p = o[axis];
    int q[3] = {o[0], o[1], o[2]};
    double acc = 0.0;
    auto tap = [&](int c, double w) {
      q[axis] = c;
      acc += w * pass_in<T, N, NT>(g, it, src_mode, io, q[0], q[1], q[2]);
    };
    if constexpr (filter == F_REFINE) {
      if ((p & 1) == 0) {
        tap(floordiv(p, 2), 1.0);
      } else {
        const int k = floordiv(p - 1, 2);
#pragma unroll
        for (int j = 0; j < N; ++j) tap(k + j + DD<N>::J0, DD<N>::w(j));
      }
    } else if constexpr (filter == F_RESTRICT) {
#pragma unroll
      for (int d = -Ha<N, NT>::R; d <= Ha<N, NT>::R; ++d)
        if (Ha<N, NT>::c(d) != 0.0) tap(2 * p + d, Ha<N, NT>::c(d));
    } else if constexpr (filter == F_SYNTH) {
      if ((p & 1) == 0) {
#pragma unroll
        for (int d = -Js<N, NT>::R; d <= Js<N, NT>::R; ++d)
          if (Js<N, NT>::c(d) != 0.0) tap(p + d, Js<N, NT>::c(d));
      } else {
#pragma unroll
        for (int d = -Ks<N, NT>::R; d <= Ks<N, NT>::R; ++d)
          if (Ks<N, NT>::c(d) != 0.0) tap(p + d, Ks<N, NT>::c(d));
      }
    } else {  // F_ANALYSIS
      if ((p & 1) == 0) {
#pragma unroll
        for (int d = -Ha<N, NT>::R; d <= Ha<N, NT>::R; ++d)
          if (Ha<N, NT>::c(d) != 0.0) tap(p + d, Ha<N, NT>::c(d));
      } else {
#pragma unroll
        for (int d = -Ga<N>::R; d <= Ga<N>::R; ++d)
          if (Ga<N>::c(d) != 0.0) tap(p + d, Ga<N>::c(d));
      }
    }
    if (dst_mode == 0) {
      io.dout[it.out_off + ((int64_t)(o[2] - it.lo[2]) * sz[1] + (o[1] - it.lo[1])) * sz[0] +
              (o[0] - it.lo[0])] = acc;
    } else {
      const int lx = o[0] - it.dlo[0], ly = o[1] - it.dlo[1], lz = o[2] - it.dlo[2];
      if ((unsigned)lx >= (unsigned)nb || (unsigned)ly >= (unsigned)nb || (unsigned)lz >= (unsigned)nb) {
        atomicAdd(g.err, 1);
        continue;
      }
      T* d = io.dst + it.dst_blk * nb3 + ((int64_t)lz * nb + ly) * nb + lx;
      if (dst_mode == 1) *d = T(acc);
      else *d = T(double(*d) - acc);
    }
  }
}

// ------------------------------------------------------------- utilities
__device__ __forceinline__ double ic_value(const IcDev& ic, double X, double Y, double Z) {
  double v = 0.0;
  if (ic.kind == 0) {
    for (int k = 0; k < ic.n; ++k) {
      const double* p = ic.params + 5 * k;
      double dx = X - p[0], dy = Y - p[1], dz = Z - p[2];
      dx -= round(dx);
      dy -= round(dy);
      dz -= round(dz);
      v += p[4] * exp(-(dx * dx + dy * dy + dz * dz) / (p[3] * p[3]));
    }
  } else {
    const double* p = ic.params;
    const double ax = (X - 0.5) / p[0], ay = (Y - 0.5) / p[1], az = (Z - 0.5) / p[2];
    const double rho = sqrt(ax * ax + ay * ay + az * az);
    const double amin = fmin(p[0], fmin(p[1], p[2]));
    v = 0.5 * (1.0 - tanh((rho - 1.0) * amin / p[3]));
  }
  return v;
}

template <typename T>
__global__ void k_sample_ic(DevGrid<T> g, IcDev ic) {
  const int nb = g.nb;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  const int64_t total = nb3 * g.nblk;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = int(i / nb3);
    const int r = int(i % nb3);
    const int x = r % nb, y = (r / nb) % nb, z = r / (nb * nb);
    const double den = double(nb << g.lev[b]);
    g.field[i] = T(ic_value(ic, double(g.ijk[3 * b] * nb + x) / den,
                            double(g.ijk[3 * b + 1] * nb + y) / den,
                            double(g.ijk[3 * b + 2] * nb + z) / den));
  }
}

// Block sums of 256 threads' FP64 partials (fixed order: deterministic).
template <int K>
__device__ __forceinline__ void block_sum(double (&s)[K], double (*red)[256]) {
  for (int k = 0; k < K; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
}

// Per-block moment partials out[4 b + k] (the host adds the blocks with a
// compensated sum, so the result does not depend on the launch order).
template <typename T>
__global__ __launch_bounds__(256) void k_moments(DevGrid<T> g, double* out) {
  __shared__ double red[4][256];
  const int b = blockIdx.x;
  const int nb = g.nb;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  const double den = double(nb << g.lev[b]);
  const double w = 1.0 / (den * den * den);
  double s[4] = {0, 0, 0, 0};
  for (int r = threadIdx.x; r < nb3; r += blockDim.x) {
    const int x = r % nb, y = (r / nb) % nb, z = r / (nb * nb);
    const double v = double(g.field[b * nb3 + r]);
    s[0] += v;
    s[1] += v * (double(g.ijk[3 * b] * nb + x) / den);
    s[2] += v * (double(g.ijk[3 * b + 1] * nb + y) / den);
    s[3] += v * (double(g.ijk[3 * b + 2] * nb + z) / den);
  }
  block_sum<4>(s, red);
  if (threadIdx.x < 4) out[4 * (int64_t)b + threadIdx.x] = w * red[threadIdx.x][0];
}

// Per-block distance to the analytic field: out[2 b] = max |phi - f|,
// out[2 b + 1] = sum h^3 (phi - f)^2, f evaluated in FP64 at the points.
template <typename T>
__global__ __launch_bounds__(256) void k_ic_error(DevGrid<T> g, IcDev ic, double* out) {
  __shared__ double red[1][256];
  __shared__ double mx[256];
  const int b = blockIdx.x;
  const int nb = g.nb;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  const double den = double(nb << g.lev[b]);
  double s[1] = {0.0};
  double m = 0.0;
  for (int r = threadIdx.x; r < nb3; r += blockDim.x) {
    const int x = r % nb, y = (r / nb) % nb, z = r / (nb * nb);
    const double f = ic_value(ic, double(g.ijk[3 * b] * nb + x) / den,
                              double(g.ijk[3 * b + 1] * nb + y) / den,
                              double(g.ijk[3 * b + 2] * nb + z) / den);
    const double e = double(g.field[b * nb3 + r]) - f;
    s[0] += e * e;
    m = fmax(m, fabs(e));
  }
  mx[threadIdx.x] = m;
  block_sum<1>(s, red);
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * (int64_t)b] = mx[0];
    out[2 * (int64_t)b + 1] = red[0][0] / (den * den * den);
  }
}

template <typename T>
__global__ void k_gather_ext(DevGrid<T> g, int depth, int64_t b0, int64_t nblk, T* out) {
  const int nb = g.nb;
  const int e = nb + 2 * depth;
  const int64_t e3 = (int64_t)e * e * e;
  const int64_t total = e3 * nblk;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = int(b0 + i / e3);
    const int r = int(i % e3);
    const int x = r % e - depth, y = (r / e) % e - depth, z = r / (e * e) - depth;
    out[i] = ext_value(g, b, x, y, z);
  }
}

template <typename T>
__global__ void k_copy_blocks(const T* __restrict__ src, T* __restrict__ dst,
                              const int32_t* __restrict__ pairs, int nb3) {
  const int dst_b = pairs[2 * blockIdx.x], src_b = pairs[2 * blockIdx.x + 1];
  for (int i = threadIdx.x; i < nb3; i += blockDim.x)
    dst[(int64_t)dst_b * nb3 + i] = src[(int64_t)src_b * nb3 + i];
}

template <typename T>
__global__ void k_fill(T* dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = T(0);
}

// ------------------------------------------------- static detail scratch
// Band maxima of the detail pass (27 doubles per block) for callers that
// cannot allocate: a file-scope device array, one copy per GPU, shared by
// every call on that GPU.  Host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's name
// (which on the host is only a stand-in).
static constexpr int64_t kStaticBandBlocks = 65536;
static __device__ __align__(256) double scratch[27 * kStaticBandBlocks];

int64_t static_band_blocks() { return kStaticBandBlocks; }

hipError_t static_band_scratch(double** out) {
  static double* ptr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}

// ------------------------------------------------------------- launchers
#define MR_WAVELET_SWITCH(w, CALL)                                   \
  do {                                                               \
    if (w.N == 2 && w.Nt == 0) { constexpr int N_ = 2, NT_ = 0; CALL; } \
    else if (w.N == 4 && w.Nt == 0) { constexpr int N_ = 4, NT_ = 0; CALL; } \
    else if (w.N == 6 && w.Nt == 0) { constexpr int N_ = 6, NT_ = 0; CALL; } \
    else if (w.N == 2 && w.Nt == 2) { constexpr int N_ = 2, NT_ = 2; CALL; } \
    else if (w.N == 4 && w.Nt == 2) { constexpr int N_ = 4, NT_ = 2; CALL; } \
    else { constexpr int N_ = 6, NT_ = 2; CALL; }                    \
  } while (0)

template <typename T, int NB>
static void gview_nb(const DevGrid<T>& g, Wavelet w, const GItem* items, int n, int lds, hipStream_t s) {
  MR_WAVELET_SWITCH(w, MR_LAUNCH((k_gview<T, N_, NT_, NB>), dim3(n), dim3(256), lds, s, g, items));
}
template <typename T>
static void gview_t(const void* dg, Wavelet w, const GItem* items, int n, int lds, hipStream_t s) {
  const DevGrid<T>& g = *static_cast<const DevGrid<T>*>(dg);
  if (g.nb == 8) gview_nb<T, 8>(g, w, items, n, lds, s);
  else if (g.nb == 16) gview_nb<T, 16>(g, w, items, n, lds, s);
  else gview_nb<T, 24>(g, w, items, n, lds, s);
}
void launch_gview(bool f32, const void* dg, Wavelet w, const GItem* items, int n, int lds,
                  hipStream_t s) {
  if (n <= 0) return;
  if (f32) gview_t<float>(dg, w, items, n, lds, s);
  else gview_t<double>(dg, w, items, n, lds, s);
}

template <typename T, int NB>
static void subst_nb(const DevGrid<T>& g, Wavelet w, const GItem* items, int n, int lds,
                     int threads, hipStream_t s) {
  if (threads == 256)
    MR_WAVELET_SWITCH(w, MR_LAUNCH((k_subst<T, N_, NT_, NB, 256>), dim3(n), dim3(256), lds, s, g,
                                   items));
  else
    MR_WAVELET_SWITCH(w, MR_LAUNCH((k_subst<T, N_, NT_, NB, 512>), dim3(n), dim3(512), lds, s, g,
                                   items));
}
template <typename T>
static void subst_t(const void* dg, Wavelet w, const GItem* items, int n, int lds, int threads,
                    hipStream_t s) {
  const DevGrid<T>& g = *static_cast<const DevGrid<T>*>(dg);
  if (g.nb == 8) subst_nb<T, 8>(g, w, items, n, lds, threads, s);
  else if (g.nb == 16) subst_nb<T, 16>(g, w, items, n, lds, threads, s);
  else subst_nb<T, 24>(g, w, items, n, lds, threads, s);
}
void launch_subst(bool f32, const void* dg, Wavelet w, const GItem* items, int n, int lds,
                  int threads, hipStream_t s) {
  if (n <= 0) return;
  if (f32) subst_t<float>(dg, w, items, n, lds, threads, s);
  else subst_t<double>(dg, w, items, n, lds, threads, s);
}

template <typename T, int NB>
static void ctab_nb(const DevGrid<T>& g, int n, hipStream_t s) {
  const int64_t th = (int64_t)n * 64;
  MR_LAUNCH((k_cell_tables<T, NB>), dim3(unsigned((th + 255) / 256)), dim3(256), 0, s, g,
            const_cast<int64_t*>(g.cbase), const_cast<int32_t*>(g.cstep), n);
}
void launch_cell_tables(bool f32, const void* dg, int n, hipStream_t s) {
  if (n <= 0) return;
  if (f32) {
    const DevGrid<float>& g = *static_cast<const DevGrid<float>*>(dg);
    if (g.nb == 8) ctab_nb<float, 8>(g, n, s);
    else if (g.nb == 16) ctab_nb<float, 16>(g, n, s);
    else ctab_nb<float, 24>(g, n, s);
  } else {
    const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dg);
    if (g.nb == 8) ctab_nb<double, 8>(g, n, s);
    else if (g.nb == 16) ctab_nb<double, 16>(g, n, s);
    else ctab_nb<double, 24>(g, n, s);
  }
}

// MAXQ bounds the coarse points per column of pass 1 (the item's extent
// along y or z, whichever is thinner): 3, 6 or 12.
template <typename T, int NB>
static void rview_nb(const DevGrid<T>& g, Wavelet w, const RItem* items, int n, int lds, int maxq,
                     hipStream_t s) {
  if (maxq <= 3)
    MR_WAVELET_SWITCH(w, MR_LAUNCH((k_restrict<T, N_, NT_, NB, 3>), dim3(n), dim3(256), lds, s, g, items));
  else if (maxq <= 6)
    MR_WAVELET_SWITCH(w, MR_LAUNCH((k_restrict<T, N_, NT_, NB, 6>), dim3(n), dim3(256), lds, s, g, items));
  else
    MR_WAVELET_SWITCH(w, MR_LAUNCH((k_restrict<T, N_, NT_, NB, 12>), dim3(n), dim3(256), lds, s, g, items));
}
template <typename T>
static void rview_t(const void* dg, Wavelet w, const RItem* items, int n, int lds, int maxq,
                    hipStream_t s) {
  const DevGrid<T>& g = *static_cast<const DevGrid<T>*>(dg);
  if (g.nb == 8) rview_nb<T, 8>(g, w, items, n, lds, maxq, s);
  else if (g.nb == 16) rview_nb<T, 16>(g, w, items, n, lds, maxq, s);
  else rview_nb<T, 24>(g, w, items, n, lds, maxq, s);
}
void launch_rview(bool f32, const void* dg, Wavelet w, const RItem* items, int n, int lds, int maxq,
                  hipStream_t s) {
  if (n <= 0) return;
  if (f32) rview_t<float>(dg, w, items, n, lds, maxq, s);
  else rview_t<double>(dg, w, items, n, lds, maxq, s);
}

template <typename T, int FD, int NB>
static void rhs_nb(const DevGrid<T>& g, const void* un, void* out, double a, double b, double c,
                   double dt, const VelDev& v, int first, int n, hipStream_t s) {
  const int nxcd = (n >= 64) ? 8 : 1;
  MR_LAUNCH((k_rhs<T, FD, NB>), dim3(n), dim3(NB * NB), 0, s, g, static_cast<const T*>(un),
            static_cast<T*>(out), T(a), T(b), T(c), T(dt), v, first, nxcd);
}
template <typename T>
static void rhs_t(const void* dgv, const void* un, void* out, int fd, double a, double b, double c,
                  double dt, const VelDev& v, int first, int n, hipStream_t s) {
  const DevGrid<T>& g = *static_cast<const DevGrid<T>*>(dgv);
  if (fd == 3) {
    if (g.nb == 8) rhs_nb<T, 3, 8>(g, un, out, a, b, c, dt, v, first, n, s);
    else if (g.nb == 16) rhs_nb<T, 3, 16>(g, un, out, a, b, c, dt, v, first, n, s);
    else rhs_nb<T, 3, 24>(g, un, out, a, b, c, dt, v, first, n, s);
  } else if (fd == 5) {
    if (g.nb == 8) rhs_nb<T, 5, 8>(g, un, out, a, b, c, dt, v, first, n, s);
    else if (g.nb == 16) rhs_nb<T, 5, 16>(g, un, out, a, b, c, dt, v, first, n, s);
    else rhs_nb<T, 5, 24>(g, un, out, a, b, c, dt, v, first, n, s);
  } else if (fd == 4) {
    if (g.nb == 8) rhs_nb<T, 4, 8>(g, un, out, a, b, c, dt, v, first, n, s);
    else if (g.nb == 16) rhs_nb<T, 4, 16>(g, un, out, a, b, c, dt, v, first, n, s);
    else rhs_nb<T, 4, 24>(g, un, out, a, b, c, dt, v, first, n, s);
  } else if (fd == 2) {
    if (g.nb == 8) rhs_nb<T, 2, 8>(g, un, out, a, b, c, dt, v, first, n, s);
    else if (g.nb == 16) rhs_nb<T, 2, 16>(g, un, out, a, b, c, dt, v, first, n, s);
    else rhs_nb<T, 2, 24>(g, un, out, a, b, c, dt, v, first, n, s);
  } else {
    if (g.nb == 8) rhs_nb<T, 6, 8>(g, un, out, a, b, c, dt, v, first, n, s);
    else if (g.nb == 16) rhs_nb<T, 6, 16>(g, un, out, a, b, c, dt, v, first, n, s);
    else rhs_nb<T, 6, 24>(g, un, out, a, b, c, dt, v, first, n, s);
  }
}
void launch_rhs(bool f32, const void* dg, const void* un, void* out, int fd, int depth, double a,
                double b, double c, double dt, const VelDev& v, int first, int n, hipStream_t s) {
  (void)depth;
  if (n <= 0) return;
  if (f32) rhs_t<float>(dg, un, out, fd, a, b, c, dt, v, first, n, s);
  else rhs_t<double>(dg, un, out, fd, a, b, c, dt, v, first, n, s);
}

template <typename T, int NB>
static void details_nb(const DevGrid<T>& g, Wavelet w, int ef, int eb, double* bands,
                       const int32_t* slot, double* det, int first, int n, hipStream_t s) {
  MR_WAVELET_SWITCH(w, MR_LAUNCH((k_details<T, NB, N_, NT_>), dim3(n), dim3(NB * NB), 0, s, g, ef,
                                 eb, bands, slot, det, first));
}
void launch_details(bool f32, const void* dgv, Wavelet w, int ef, int eb, double* bands,
                    const int32_t* slot, double* det, int first, int n, hipStream_t s) {
  if (n <= 0) return;
  if (f32) {
    const DevGrid<float>& g = *static_cast<const DevGrid<float>*>(dgv);
    if (g.nb == 8) details_nb<float, 8>(g, w, ef, eb, bands, slot, det, first, n, s);
    else if (g.nb == 16) details_nb<float, 16>(g, w, ef, eb, bands, slot, det, first, n, s);
    else details_nb<float, 24>(g, w, ef, eb, bands, slot, det, first, n, s);
  } else {
    const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dgv);
    if (g.nb == 8) details_nb<double, 8>(g, w, ef, eb, bands, slot, det, first, n, s);
    else if (g.nb == 16) details_nb<double, 16>(g, w, ef, eb, bands, slot, det, first, n, s);
    else details_nb<double, 24>(g, w, ef, eb, bands, slot, det, first, n, s);
  }
}

void launch_combine(const void* dgv, const double* bands, int ext, double* norms, int n,
                    hipStream_t s) {
  if (n <= 0) return;
  const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dgv);  // metadata only
  hipLaunchKernelGGL(k_combine, dim3((n + 255) / 256), dim3(256), 0, s, g.lev, g.cmap, bands, ext,
                     norms, n);
}

void launch_sample_ic(bool f32, const void* dgv, const IcDev& ic, hipStream_t s) {
  if (f32) {
    const DevGrid<float>& g = *static_cast<const DevGrid<float>*>(dgv);
    hipLaunchKernelGGL(k_sample_ic<float>, dim3(2048), dim3(256), 0, s, g, ic);
  } else {
    const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dgv);
    hipLaunchKernelGGL(k_sample_ic<double>, dim3(2048), dim3(256), 0, s, g, ic);
  }
}

void launch_moments(bool f32, const void* dgv, double* out, hipStream_t s) {
  if (f32) {
    const DevGrid<float>& g = *static_cast<const DevGrid<float>*>(dgv);
    if (g.nblk) hipLaunchKernelGGL(k_moments<float>, dim3(g.nblk), dim3(256), 0, s, g, out);
  } else {
    const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dgv);
    if (g.nblk) hipLaunchKernelGGL(k_moments<double>, dim3(g.nblk), dim3(256), 0, s, g, out);
  }
}

void launch_ic_error(bool f32, const void* dgv, const IcDev& ic, double* out, hipStream_t s) {
  if (f32) {
    const DevGrid<float>& g = *static_cast<const DevGrid<float>*>(dgv);
    if (g.nblk) hipLaunchKernelGGL(k_ic_error<float>, dim3(g.nblk), dim3(256), 0, s, g, ic, out);
  } else {
    const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dgv);
    if (g.nblk) hipLaunchKernelGGL(k_ic_error<double>, dim3(g.nblk), dim3(256), 0, s, g, ic, out);
  }
}

void launch_gather_ext(bool f32, const void* dgv, int depth, int64_t b0, int64_t nblk, void* out,
                       hipStream_t s) {
  if (nblk <= 0) return;
  if (f32) {
    const DevGrid<float>& g = *static_cast<const DevGrid<float>*>(dgv);
    hipLaunchKernelGGL(k_gather_ext<float>, dim3(1024), dim3(256), 0, s, g, depth, b0, nblk,
                       static_cast<float*>(out));
  } else {
    const DevGrid<double>& g = *static_cast<const DevGrid<double>*>(dgv);
    hipLaunchKernelGGL(k_gather_ext<double>, dim3(1024), dim3(256), 0, s, g, depth, b0, nblk,
                       static_cast<double*>(out));
  }
}

void launch_copy_blocks(bool f32, const void* src, void* dst, const int32_t* pairs, int n, int nb,
                        hipStream_t s) {
  if (n <= 0) return;
  const int nb3 = nb * nb * nb;
  if (f32)
    hipLaunchKernelGGL(k_copy_blocks<float>, dim3(n), dim3(256), 0, s,
                       static_cast<const float*>(src), static_cast<float*>(dst), pairs, nb3);
  else
    hipLaunchKernelGGL(k_copy_blocks<double>, dim3(n), dim3(256), 0, s,
                       static_cast<const double*>(src), static_cast<double*>(dst), pairs, nb3);
}

void launch_fill(bool f32, void* dst, size_t n, hipStream_t s) {
  if (n == 0) return;
  if (f32) hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, static_cast<float*>(dst), n);
  else hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, static_cast<double*>(dst), n);
}

template <typename T>
static void pass_t(const void* dgv, Wavelet w, int filter, int axis, int src_mode, int dst_mode,
                   const PItem* items, int n, const double* din, double* dout, const double* det,
                   const int32_t* slot, const uint32_t* tab, void* dst, hipStream_t s) {
  const DevGrid<T>& g = *static_cast<const DevGrid<T>*>(dgv);
  PassIO<T> io{din, dout, det, slot, tab, static_cast<T*>(dst)};
#define MR_PASS(F, S)                                                                    \
  MR_WAVELET_SWITCH(w, hipLaunchKernelGGL((k_pass<T, N_, NT_, F, S>), dim3(n), dim3(256), 0, s, \
                                          g, items, axis, dst_mode, io))
  // the (filter, source) pairs the adaptation uses: each filter's first
  // pass reads the field (refine, restrict) or the discarded details
  // (synthesis), later passes the scratch box
  if (filter == F_REFINE && src_mode == 0) MR_PASS(F_REFINE, 0);
  else if (filter == F_REFINE) MR_PASS(F_REFINE, 1);
  else if (filter == F_RESTRICT && src_mode == 0) MR_PASS(F_RESTRICT, 0);
  else if (filter == F_RESTRICT) MR_PASS(F_RESTRICT, 1);
  else if (filter == F_SYNTH && src_mode == 2) MR_PASS(F_SYNTH, 2);
  else if (filter == F_SYNTH) MR_PASS(F_SYNTH, 1);
  else if (src_mode == 0) MR_PASS(F_ANALYSIS, 0);
  else MR_PASS(F_ANALYSIS, 1);
#undef MR_PASS
}
void launch_pass(bool f32, const void* dgv, Wavelet w, int filter, int axis, int src_mode,
                 int dst_mode, const PItem* items, int n, const double* din, double* dout,
                 const double* det, const int32_t* slot, const uint32_t* tab, void* dst,
                 hipStream_t s) {
  if (n <= 0) return;
  if (f32)
    pass_t<float>(dgv, w, filter, axis, src_mode, dst_mode, items, n, din, dout, det, slot, tab, dst, s);
  else
    pass_t<double>(dgv, w, filter, axis, src_mode, dst_mode, items, n, din, dout, det, slot, tab, dst, s);
}

}  // namespace mr
