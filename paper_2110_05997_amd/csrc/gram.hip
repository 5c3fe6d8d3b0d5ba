// Mode-l unfolding Gram G_l = T_(l) T_(l)^T on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// The left singular vectors of T_(l) are the eigenvectors of this Gram (App. B lemma on the SVD of
// M and the eigenvectors of M M^T); computing it is the dominant cost of the classic truncated
// MLSVD (ch.2 MLSVD cost discussion, ch.4 Alg. Compression).  The Gram does not depend on the
// ordering of the unfolding's columns, so the three modes are read straight from the C-ordered
// tensor T[i1][i2][i3]:
//   mode 1: rows m = i1 of the I1 x (I2 I3) matrix            (contraction index contiguous)
//   mode 2: sum over i1 of the I2 x I3 slab T[i1] times its transpose (contraction contiguous)
//   mode 3: columns of the (I1 I2) x I3 matrix                 (rows m contiguous)
// FP32 input is promoted exactly to FP64 before the MFMA, so all three precisions accumulate in
// FP64.  Work split: 64x64 tiles of the upper triangle of G times split-K chunks; each workgroup
// writes a partial tile and a second kernel sums the partials in a fixed order (bit-reproducible).
#include "common.h"

namespace cpd {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 64;   // G tile edge
constexpr int BK = 32;     // contraction chunk staged in LDS
constexpr int NT = 256;    // 4 waves, each a 32x32 quarter of the tile
constexpr int LDP = BK + 1;

struct GramGeom {
  int variant;        // 0: rows (modes 1, 2), 1: columns (mode 3)
  int M;              // Gram size
  long long Ktot;     // total contraction length (B*K for variant 0)
  long long K;        // inner contraction length of one slab (variant 0)
  long long sb, sm;   // variant 0: slab stride, row stride
  long long sk;       // variant 1: row stride of the (I1 I2) x I3 view
  int ntile;          // tiles per edge
  int nupper;         // number of upper-triangle tiles
  int nsplit;         // split-K factor (multiple of 8)
  long long kchunk;   // contraction length per split (multiple of BK)
};

template <class T>
__device__ __forceinline__ double ld(const T* p, long long i) { return (double)p[i]; }
template <>
__device__ __forceinline__ double ld<uint16_t>(const uint16_t* p, long long i) { return bf16_bits_to_f64(p[i]); }

__device__ __forceinline__ void tile_of(int t, int ntile, int& tm, int& tn) {
  int row = 0, start = 0;
  while (t >= start + (ntile - row)) { start += ntile - row; ++row; }
  tm = row;
  tn = row + (t - start);
}

template <class T>
__device__ __forceinline__ void stage(double (*X)[LDP], const T* __restrict__ src, const GramGeom& g,
                                      int row0, long long k0, long long kend) {
  const int tid = threadIdx.x;
  if (g.variant == 0) {
#pragma unroll
    for (int t = 0; t < (TILE * BK) / NT; ++t) {
      const int e = tid + t * NT;
      const int kk = e % BK, m = e / BK;
      const long long kp = k0 + kk;
      const int gm = row0 + m;
      double v = 0.0;
      if (gm < g.M && kp < kend) {
        const long long b = kp / g.K, k = kp - b * g.K;
        v = ld(src, b * g.sb + (long long)gm * g.sm + k);
      }
      X[m][kk] = v;
    }
  } else {
#pragma unroll
    for (int t = 0; t < (TILE * BK) / NT; ++t) {
      const int e = tid + t * NT;
      const int m = e % TILE, kk = e / TILE;
      const long long kp = k0 + kk;
      const int gm = row0 + m;
      double v = 0.0;
      if (gm < g.M && kp < kend) v = ld(src, kp * g.sk + gm);
      X[m][kk] = v;
    }
  }
}

template <class T>
__global__ __launch_bounds__(NT) void gram_partial_kernel(const T* __restrict__ src, GramGeom g,
                                                          double* __restrict__ part) {
  __shared__ double Xm[TILE][LDP];
  __shared__ double Xn[TILE][LDP];
  // XCD-aware order: workgroup L runs on XCD L % 8.  Consecutive workgroups of one XCD take all
  // tiles of one split, so the rows of that contraction chunk are reused from the XCD's L2.
  const int L = blockIdx.x;
  const int xcd = L & 7, idx = L >> 3;
  const int tile = idx % g.nupper;
  const int split = (idx / g.nupper) * 8 + xcd;
  if (split >= g.nsplit) return;
  int tm, tn;
  tile_of(tile, g.ntile, tm, tn);
  const bool diag = (tm == tn);
  const long long kbeg = (long long)split * g.kchunk;
  const long long kend = min(g.Ktot, kbeg + g.kchunk);

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  double (*Bn)[LDP] = diag ? Xm : Xn;
  for (long long k0 = kbeg; k0 < kend; k0 += BK) {
    stage(Xm, src, g, tm * TILE, k0, kend);
    if (!diag) stage(Xn, src, g, tn * TILE, k0, kend);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      // A fragment: lane holds A[lane%16][lane/16] (16x4); B fragment: B[lane/16][lane%16] (4x16)
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Xm[wm + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bn[wn + 16 * j + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[4*v + lane/16][lane%16] lives in acc[..][v] (result layout of v_mfma_f64_16x16x4f64)
  double* out = part + ((long long)tile * g.nsplit + split) * (TILE * TILE);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wm + 16 * i + 4 * v + (lane >> 4);
        const int c = wn + 16 * j + (lane & 15);
        out[r * TILE + c] = acc[i][j][v];
      }
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, GramGeom g, double* __restrict__ G) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)g.nupper * TILE * TILE) return;
  const int tile = (int)(e / (TILE * TILE));
  const int rc = (int)(e % (TILE * TILE));
  const int r = rc / TILE, c = rc % TILE;
  int tm, tn;
  tile_of(tile, g.ntile, tm, tn);
  if (tm == tn && r > c) return;
  const int m = tm * TILE + r, n = tn * TILE + c;
  if (m >= g.M || n >= g.M) return;
  const double* p = part + (long long)tile * g.nsplit * (TILE * TILE) + rc;
  double s = 0.0;
  for (int k = 0; k < g.nsplit; ++k) s += p[(long long)k * TILE * TILE];
  G[(long long)m * g.M + n] = s;
  G[(long long)n * g.M + m] = s;
}

GramGeom make_geom(const int64_t dims[3], int mode) {
  GramGeom g{};
  const long long I1 = dims[0], I2 = dims[1], I3 = dims[2];
  if (mode == 0) {
    g.variant = 0; g.M = (int)I1; g.K = I2 * I3; g.Ktot = g.K; g.sb = 0; g.sm = I2 * I3;
  } else if (mode == 1) {
    g.variant = 0; g.M = (int)I2; g.K = I3; g.Ktot = I1 * I3; g.sb = I2 * I3; g.sm = I3;
  } else {
    g.variant = 1; g.M = (int)I3; g.Ktot = I1 * I2; g.sk = I3;
  }
  g.ntile = (g.M + TILE - 1) / TILE;
  g.nupper = g.ntile * (g.ntile + 1) / 2;
  // aim for ~1024 workgroups (4 per CU) without chunks shorter than 4*BK
  long long want = (1024 + g.nupper - 1) / g.nupper;
  long long maxsplit = (g.Ktot + 4 * BK - 1) / (4 * BK);
  long long ns = want < maxsplit ? want : maxsplit;
  if (ns < 1) ns = 1;
  ns = (ns + 7) / 8 * 8;
  long long chunk = (g.Ktot + ns - 1) / ns;
  chunk = (chunk + BK - 1) / BK * BK;
  ns = (g.Ktot + chunk - 1) / chunk;
  ns = (ns + 7) / 8 * 8;
  g.nsplit = (int)ns;
  g.kchunk = chunk;
  return g;
}

}  // namespace

size_t gram_ws_bytes(const int64_t dims[3], int mode) {
  GramGeom g = make_geom(dims, mode);
  return align_up((size_t)g.nupper * g.nsplit * TILE * TILE * sizeof(double), 256);
}

cpd_status gram(const void* T, int dtype, const int64_t dims[3], int mode, int compute_dtype,
                double* G, void* ws, size_t ws_bytes, hipStream_t s) {
  (void)compute_dtype;
  if (mode < 0 || mode > 2 || T == nullptr || G == nullptr) {
    set_error("gram: bad arguments");
    return CPD_E_INVALID;
  }
  GramGeom g = make_geom(dims, mode);
  const size_t need = gram_ws_bytes(dims, mode);
  if (ws == nullptr || ws_bytes < need) {
    set_error("gram: workspace %zu < %zu", ws_bytes, need);
    return CPD_E_WORKSPACE;
  }
  double* part = (double*)ws;
  const int nblocks = g.nupper * g.nsplit;
  prof_begin(CPD_PK_GRAM, s);
  switch (dtype) {
    case CPD_F64:
      hipLaunchKernelGGL(gram_partial_kernel<double>, dim3(nblocks), dim3(NT), 0, s,
                         (const double*)T, g, part);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(gram_partial_kernel<float>, dim3(nblocks), dim3(NT), 0, s,
                         (const float*)T, g, part);
      break;
    case CPD_BF16:
      hipLaunchKernelGGL(gram_partial_kernel<uint16_t>, dim3(nblocks), dim3(NT), 0, s,
                         (const uint16_t*)T, g, part);
      break;
    default:
      set_error("gram: bad dtype %d", dtype);
      return CPD_E_INVALID;
  }
  prof_end(CPD_PK_GRAM, s);
  CPD_LAUNCH_CHECK();
  const long long nel = (long long)g.nupper * TILE * TILE;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s,
                     part, g, G);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
