// Full-tensor MTTKRP M_l = T_(l) (W^(c) (.) W^(b)), the contraction behind the gradient of ch.3
// Lemma gradF / ch.4 dGN when it runs on the uncompressed tensor:
//   M_l[m][r] = sum over the other two indices (x, y) of T[...] Wa[x][r] Wb[y][r].
// One FP64 MFMA (16x16x4) GEMM per mode with the Khatri-Rao operand formed on the fly:
//  * the contraction runs over (x, y), the two other modes (y the faster in memory for modes 1 and
//    2, the slower for mode 3); a workgroup owns 64 output rows and a range of x, and walks y in
//    32-wide tiles, so every address is a base plus an offset and no index needs a division;
//  * M[m][r] = sum_x Wa[x][r] (sum_y T[m, x, y] Wb[y][r]): per tile it stages T (converted to
//    FP64) and rows of Wb in LDS, the next tile's loads in flight during this tile's MFMAs, and
//    after the last y-tile of an x the inner sums are scaled by Wa[x] and added;
//  * each of the four waves accumulates 16 rows x ceil(R/16) 16-column tiles;
//  * chunks write partial sums that a second kernel adds in a fixed order (bit-reproducible).
#include "common.h"

namespace cpd {
namespace {

constexpr int MT_ROWS = 64;
constexpr int MT_KT = 32;
constexpr int MT_NT = 256;
constexpr int MT_MAXR = 64;

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <class TT>
__device__ __forceinline__ double tval(const TT* p) { return (double)*p; }
template <>
__device__ __forceinline__ double tval<uint16_t>(const uint16_t* p) { return bf16_bits_to_f64(*p); }

struct MtGeom {
  int I1, I2, I3;
  int rows;        // I_l
  int X, Y;        // extents of the outer and inner contraction indices
  int xper;        // outer indices per workgroup
  int R, nct;      // rank, 16-column tiles
};

// T element (row m, outer x, inner y) of the mode-MODE unfolding:
//   mode 1: T[m][x][y], mode 2: T[x][m][y], mode 3: T[x][y][m]
template <class TT, int MODE>
__device__ __forceinline__ const TT* t_ptr(const TT* T, const MtGeom& g, int m, int x, int y) {
  if (MODE == 0) return T + ((long long)m * g.I2 + x) * g.I3 + y;
  if (MODE == 1) return T + ((long long)x * g.I2 + m) * g.I3 + y;
  return T + ((long long)x * g.I2 + y) * g.I3 + m;
}

constexpr int MT_AU = MT_ROWS * MT_KT / MT_NT;    // T elements staged per thread and tile

template <class TT, int MODE, int NCT>
__global__ __launch_bounds__(MT_NT) void mttkrp_mfma_kernel(const TT* __restrict__ T, MtGeom g,
                                                            const double* __restrict__ Wa,
                                                            const double* __restrict__ Wb,
                                                            double* __restrict__ part) {
  __shared__ double As[MT_ROWS][MT_KT + 1];
  __shared__ double Bs[MT_KT][MT_MAXR + 1];
  const int rb = blockIdx.x, split = blockIdx.y;
  const int m0 = rb * MT_ROWS;
  const int xbeg = split * g.xper, xend = min(xbeg + g.xper, g.X);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int R = g.R, Y = g.Y;
  constexpr int ncol = NCT * 16;
  // T element u of this thread: (row, inner offset) = (am0 + u * amu, ak0 + u * aku); threads run
  // along the index that is contiguous in memory (y for modes 1 and 2, the row for mode 3)
  const int am0 = (MODE == 2) ? (tid & (MT_ROWS - 1)) : (tid >> 5);
  const int ak0 = (MODE == 2) ? (tid >> 6) : (tid & (MT_KT - 1));
  constexpr int amu = (MODE == 2) ? 0 : MT_NT / MT_KT;
  constexpr int aku = (MODE == 2) ? MT_NT / MT_ROWS : 0;
  constexpr int MT_BU = MT_KT * ncol / MT_NT;   // Khatri-Rao elements per thread and tile
  int bk[MT_BU], bc[MT_BU];
#pragma unroll
  for (int u = 0; u < MT_BU; ++u) {
    const int e = tid + u * MT_NT;
    bk[u] = e / ncol;
    bc[u] = e - bk[u] * ncol;
  }
  double ra[MT_AU], rbv[MT_BU];
  // loads are unconditional (indices clamped into range, values selected afterwards) so that a
  // tile's loads issue back to back instead of each waiting behind a branch
  auto fetch = [&](int x, int y0) {
#pragma unroll
    for (int u = 0; u < MT_AU; ++u) {
      const int m = m0 + am0 + u * amu, y = y0 + ak0 + u * aku;
      const bool ok = (m < g.rows) && (y < Y);
      const double v = tval(t_ptr<TT, MODE>(T, g, ok ? m : 0, x, ok ? y : 0));
      ra[u] = ok ? v : 0.0;
    }
#pragma unroll
    for (int u = 0; u < MT_BU; ++u) {
      const int y = y0 + bk[u];
      const bool ok = (bc[u] < R) && (y < Y);
      const int col = ok ? bc[u] : 0, yc = ok ? y : 0;
      const double v = Wb[yc * R + col];
      rbv[u] = ok ? v : 0.0;
    }
  };
  // acc accumulates sum_x Wa[x][r] accx, accx = sum_y T[m, x, y] Wb[y][r] for the current x; a
  // lane's accumulator entries all belong to column c * 16 + r16
  dbl4 acc[NCT], accx[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
    acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    accx[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
  int x = xbeg, y0 = 0;
  if (x < xend) fetch(x, y0);
  while (x < xend) {
#pragma unroll
    for (int u = 0; u < MT_AU; ++u) As[am0 + u * amu][ak0 + u * aku] = ra[u];
#pragma unroll
    for (int u = 0; u < MT_BU; ++u) Bs[bk[u]][bc[u]] = rbv[u];
    __syncthreads();
    // next tile: (x, y0 + KT), wrapping to the next outer index; its loads overlap the MFMAs
    int xn = x, yn = y0 + MT_KT;
    if (yn >= Y) { yn = 0; ++xn; }
    if (xn < xend) fetch(xn, yn);
    // every k-step runs (the tail of the last y-tile is zero-padded): no branch around the MFMAs
#pragma unroll
    for (int s = 0; s < MT_KT / 4; ++s) {
      const double a = As[w * 16 + r16][4 * s + kq];
#pragma unroll
      for (int c = 0; c < NCT; ++c)
        accx[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[4 * s + kq][c * 16 + r16], accx[c], 0, 0, 0);
    }
    if (xn != x) {   // last y-tile of this x: fold in Wa[x]
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int col = c * 16 + r16;
        const double wa = Wa[x * R + (col < R ? col : 0)];
        const double f = (col < R) ? wa : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[c][v] = fma(f, accx[c][v], acc[c][v]);
        accx[c] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
    }
    __syncthreads();
    x = xn;
    y0 = yn;
  }
  double* out = part + (long long)split * g.rows * R;
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + w * 16 + 4 * v + kq, col = c * 16 + r16;
      if (row < g.rows && col < R) out[(long long)row * R + col] = acc[c][v];
    }
  }
}

// M[m][r] = sum_s part[s][m][r]: eight threads per output each add every eighth split (four
// interleaved sums each, so loads stay in flight); the eight results are combined in a fixed order.
__global__ __launch_bounds__(256) void mttkrp_reduce_kernel(const double* __restrict__ part, int nsplit, long long n,
                                                            double* __restrict__ M) {
  __shared__ double red[8][33];
  const int o = threadIdx.x & 31, q = threadIdx.x >> 5;
  const long long e = (long long)blockIdx.x * 32 + o;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < n) {
    int sp = q;
    for (; sp + 24 < nsplit; sp += 32) {
      s0 += part[(long long)sp * n + e];
      s1 += part[(long long)(sp + 8) * n + e];
      s2 += part[(long long)(sp + 16) * n + e];
      s3 += part[(long long)(sp + 24) * n + e];
    }
    for (; sp < nsplit; sp += 8) s0 += part[(long long)sp * n + e];
  }
  red[q][o] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (q == 0 && e < n)
    M[e] = ((red[0][o] + red[1][o]) + (red[2][o] + red[3][o])) + ((red[4][o] + red[5][o]) + (red[6][o] + red[7][o]));
}

MtGeom mt_geom(const int64_t dims[3], int R, int mode, int* nsplit, int* rblocks) {
  MtGeom g;
  g.I1 = (int)dims[0]; g.I2 = (int)dims[1]; g.I3 = (int)dims[2];
  g.rows = (int)dims[mode];
  g.X = (mode == 0) ? g.I2 : g.I1;
  g.Y = (mode == 2) ? g.I2 : g.I3;
  g.R = R;
  g.nct = (R + 15) / 16;
  const int rbk = (g.rows + MT_ROWS - 1) / MT_ROWS;
  // about 1024 workgroups, each with at least four k-tiles of work
  const int tiles_per_x = (g.Y + MT_KT - 1) / MT_KT;
  const int want = (1024 + rbk - 1) / rbk;
  int xper = (g.X + want - 1) / want;
  const int min_x = (4 + tiles_per_x - 1) / tiles_per_x;
  if (xper < min_x) xper = min_x;
  g.xper = xper;
  *nsplit = (g.X + xper - 1) / xper;
  *rblocks = rbk;
  return g;
}

template <class TT, int MODE>
void launch_mode(const TT* t, const MtGeom& g, const double* Wa, const double* Wb, double* part, dim3 grid,
                 hipStream_t s) {
  switch (g.nct) {
    case 1: hipLaunchKernelGGL((mttkrp_mfma_kernel<TT, MODE, 1>), grid, dim3(MT_NT), 0, s, t, g, Wa, Wb, part); break;
    case 2: hipLaunchKernelGGL((mttkrp_mfma_kernel<TT, MODE, 2>), grid, dim3(MT_NT), 0, s, t, g, Wa, Wb, part); break;
    case 3: hipLaunchKernelGGL((mttkrp_mfma_kernel<TT, MODE, 3>), grid, dim3(MT_NT), 0, s, t, g, Wa, Wb, part); break;
    default: hipLaunchKernelGGL((mttkrp_mfma_kernel<TT, MODE, 4>), grid, dim3(MT_NT), 0, s, t, g, Wa, Wb, part); break;
  }
}

template <class TT>
void launch_mt(const void* T, const MtGeom& g, int mode, const double* Wa, const double* Wb, double* part,
               dim3 grid, hipStream_t s) {
  const TT* t = (const TT*)T;
  if (mode == 0) launch_mode<TT, 0>(t, g, Wa, Wb, part, grid, s);
  else if (mode == 1) launch_mode<TT, 1>(t, g, Wa, Wb, part, grid, s);
  else launch_mode<TT, 2>(t, g, Wa, Wb, part, grid, s);
}

}  // namespace

size_t mttkrp_ws_bytes(const int64_t dims[3], int R, int mode) {
  int ns, rb;
  const MtGeom g = mt_geom(dims, R, mode, &ns, &rb);
  Sizer z;
  z.take<double>((size_t)ns * g.rows * R);
  return z.off;
}

cpd_status mttkrp_full(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                       int R, int mode, double* M, void* ws, size_t ws_bytes, hipStream_t s) {
  if (R < 1 || R > MT_MAXR || mode < 0 || mode > 2 || !T || !M || !W[0] || !W[1] || !W[2]) {
    set_error("mttkrp_full: bad arguments (R=%d mode=%d)", R, mode);
    return CPD_E_INVALID;
  }
  if (!ws || ws_bytes < mttkrp_ws_bytes(dims, R, mode)) {
    set_error("mttkrp_full: workspace too small");
    return CPD_E_WORKSPACE;
  }
  int ns, rb;
  const MtGeom g = mt_geom(dims, R, mode, &ns, &rb);
  const double* Wa = W[mode == 0 ? 1 : 0];
  const double* Wb = W[mode == 2 ? 1 : 2];
  double* part = (double*)ws;
  const dim3 grid(rb, ns);
  prof_begin(CPD_PK_MTTKRP, s);
  if (dtype == CPD_F64) launch_mt<double>(T, g, mode, Wa, Wb, part, grid, s);
  else if (dtype == CPD_F32) launch_mt<float>(T, g, mode, Wa, Wb, part, grid, s);
  else launch_mt<uint16_t>(T, g, mode, Wa, Wb, part, grid, s);
  const long long n = (long long)g.rows * R;
  hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, s, part, ns, n, M);
  prof_end(CPD_PK_MTTKRP, s);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
