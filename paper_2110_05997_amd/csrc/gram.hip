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
// FP64.  Work split: tiles of the upper triangle of G (64x64; 128x128 for large modes) times split-K
// chunks; each workgroup writes a partial tile and a second kernel sums the partials in a fixed order (bit-reproducible).
#include "common.h"

namespace cpd {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 64;   // G tile edge
constexpr int NT = 256;    // 4 waves, each a 32x32 quarter of the tile

struct GramGeom {
  int variant;        // 0: rows (modes 1, 2), 1: columns (mode 3)
  int M;              // Gram size
  int Ktot;           // total contraction length (slabs x K for variant 0)
  int K;              // inner contraction length of one slab (variant 0)
  long long sb;       // variant 0: slab stride
  int sm;             // variant 0: row stride
  int sk;             // variant 1: row stride of the (I1 I2) x I3 view
  int ntile;          // tiles per edge
  int nupper;         // number of upper-triangle tiles
  int nsplit;         // split-K factor (multiple of 8)
  int kchunk;         // contraction length per split (multiple of the k-tile)
};

// Staged value of a tensor element: FP64 for the FP64 path (BF16 bits decoded), raw bits for the
// BF16 path.
template <class V, class T>
__device__ __forceinline__ V conv(T x) { return (V)x; }
template <>
__device__ __forceinline__ double conv<double, uint16_t>(uint16_t x) { return bf16_bits_to_f64(x); }

__device__ __forceinline__ void tile_of(int t, int ntile, int& tm, int& tn) {
  int row = 0, start = 0;
  while (t >= start + (ntile - row)) { start += ntile - row; ++row; }
  tm = row;
  tn = row + (t - start);
}

// Pointer to element (row gm, contraction index kp) of the unfolding; both already clamped into
// range.  Variant 0 splits kp = b K + k by a double-precision reciprocal (exact for kp < 2^26).
template <class T>
__device__ __forceinline__ const T* elem(const T* src, const GramGeom g, int gm, int kp, double invK) {
  if (g.variant == 0) {
    const int b = (int)(((double)kp + 0.5) * invK);
    const int k = kp - b * g.K;
    return src + (long long)b * g.sb + (long long)gm * g.sm + k;
  }
  return src + (long long)kp * g.sk + gm;
}

// Staging of one k-tile of the two 64-row operands: every thread owns the same (row, k) slots in
// every tile; loads are unconditional (indices clamped, values zeroed afterwards) so they issue
// back to back, and they are made for tile t + 1 while tile t is multiplied.
template <class T, class V, int BKT>
struct Stager {
  static constexpr int PER = TILE * BKT / NT;   // elements per thread and operand
  int m[PER], kk[PER];
  T rm[PER], rn[PER];   // raw loaded values: masked and converted by put(), after the MFMAs, so
                        // a select right after a load does not make each load wait for the last
  __device__ __forceinline__ void init(const GramGeom g) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + t * NT;
      if (g.variant == 0) { kk[t] = e % BKT; m[t] = e / BKT; }   // contraction index contiguous
      else { m[t] = e % TILE; kk[t] = e / TILE; }                // row index contiguous
    }
  }
  __device__ __forceinline__ void fetch(const T* src, const GramGeom g, double invK, int rowm, int rown, bool diag, int k0, int kend) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int kp = k0 + kk[t];
      const bool okk = kp < kend;
      const int kc = okk ? kp : 0;
      const int gm = rowm + m[t], gn = rown + m[t];
      const bool okm = okk && gm < g.M, okn = okk && gn < g.M;
      rm[t] = *elem(src, g, okm ? gm : 0, kc, invK);
      if (!diag) rn[t] = *elem(src, g, okn ? gn : 0, kc, invK);
    }
  }
  // staged value of slot t for the rows (rowm, rown) and contraction start k0, zero when out of range
  __device__ __forceinline__ V valm(const GramGeom g, int t, int rowm, int k0, int kend) const {
    return (rowm + m[t] < g.M && k0 + kk[t] < kend) ? conv<V, T>(rm[t]) : (V)0;
  }
  __device__ __forceinline__ V valn(const GramGeom g, int t, int rown, int k0, int kend) const {
    return (rown + m[t] < g.M && k0 + kk[t] < kend) ? conv<V, T>(rn[t]) : (V)0;
  }
};

// FP64 path (FP64 / FP32 input promoted exactly): v_mfma_f64_16x16x4f64, 32-wide k-tiles.
constexpr int BK = 32;
constexpr int LDP = BK + 1;

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
  const int kbeg = split * g.kchunk;
  const int kend = min(g.Ktot, kbeg + g.kchunk);
  const double invK = 1.0 / (double)(g.variant == 0 ? g.K : 1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  Stager<T, double, BK> st;
  st.init(g);
  double (*Bn)[LDP] = diag ? Xm : Xn;
  if (kbeg < kend) st.fetch(src, g, invK, tm * TILE, tn * TILE, diag, kbeg, kend);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int t = 0; t < st.PER; ++t) {
      Xm[st.m[t]][st.kk[t]] = st.valm(g, t, tm * TILE, k0, kend);
      if (!diag) Xn[st.m[t]][st.kk[t]] = st.valn(g, t, tn * TILE, k0, kend);
    }
    __syncthreads();
    if (k0 + BK < kend) st.fetch(src, g, invK, tm * TILE, tn * TILE, diag, k0 + BK, kend);
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

// BF16 path: v_mfma_f32_16x16x16bf16_1k with FP32 accumulation inside a split (the split sums
// are added in FP64), 64-wide k-tiles.  Fragment layout (checked on the device): A[i][k] is
// element k % 4 of lane i + 16 (k / 4), B[k][j] element k % 4 of lane j + 16 (k / 4), and
// D[4 (l / 16) + v][l % 16] is acc[v] of lane l.
constexpr int BKH = 64;
constexpr int LDH = BKH + 4;   // row pitch in bf16 elements (keeps 8-byte fragment reads aligned)

__global__ __launch_bounds__(NT) void gram_partial_bf16_kernel(const uint16_t* __restrict__ src, GramGeom g,
                                                               double* __restrict__ part) {
  __shared__ __align__(16) uint16_t Hm[TILE][LDH];
  __shared__ __align__(16) uint16_t Hn[TILE][LDH];
  const int L = blockIdx.x;
  const int xcd = L & 7, idx = L >> 3;
  const int tile = idx % g.nupper;
  const int split = (idx / g.nupper) * 8 + xcd;
  if (split >= g.nsplit) return;
  int tm, tn;
  tile_of(tile, g.ntile, tm, tn);
  const bool diag = (tm == tn);
  const int kbeg = split * g.kchunk;
  const int kend = min(g.Ktot, kbeg + g.kchunk);
  const double invK = 1.0 / (double)(g.variant == 0 ? g.K : 1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  flt4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  Stager<uint16_t, uint16_t, BKH> st;
  st.init(g);
  uint16_t (*Bn)[LDH] = diag ? Hm : Hn;
  if (kbeg < kend) st.fetch(src, g, invK, tm * TILE, tn * TILE, diag, kbeg, kend);
  for (int k0 = kbeg; k0 < kend; k0 += BKH) {
#pragma unroll
    for (int t = 0; t < st.PER; ++t) {
      Hm[st.m[t]][st.kk[t]] = st.valm(g, t, tm * TILE, k0, kend);
      if (!diag) Hn[st.m[t]][st.kk[t]] = st.valn(g, t, tn * TILE, k0, kend);
    }
    __syncthreads();
    if (k0 + BKH < kend) st.fetch(src, g, invK, tm * TILE, tn * TILE, diag, k0 + BKH, kend);
#pragma unroll
    for (int kk = 0; kk < BKH; kk += 16) {
      bf16x4 a[2], b[2];
      const int kq = kk + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *(const bf16x4*)&Hm[wm + 16 * i + (lane & 15)][kq];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *(const bf16x4*)&Bn[wn + 16 * j + (lane & 15)][kq];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + ((long long)tile * g.nsplit + split) * (TILE * TILE);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wm + 16 * i + 4 * (lane >> 4) + v;   // bf16 result layout differs from f64's
        const int c = wn + 16 * j + (lane & 15);
        out[r * TILE + c] = (double)acc[i][j][v];
      }
}

template <int TE>
__global__ void gram_reduce_kernel(const double* __restrict__ part, GramGeom g, double* __restrict__ G) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)g.nupper * TE * TE) return;
  const int tile = (int)(e / (TE * TE));
  const int rc = (int)(e % (TE * TE));
  const int r = rc / TE, c = rc % TE;
  int tm, tn;
  tile_of(tile, g.ntile, tm, tn);
  if (tm == tn && r > c) return;
  const int m = tm * TE + r, n = tn * TE + c;
  if (m >= g.M || n >= g.M) return;
  const double* p = part + (long long)tile * g.nsplit * (TE * TE) + rc;
  double s = 0.0;
  // sixteen loads in flight per thread; the additions stay in split order
#pragma unroll 16
  for (int k = 0; k < g.nsplit; ++k) s += p[(long long)k * TE * TE];
  G[(long long)m * g.M + n] = s;
  G[(long long)n * g.M + m] = s;
}

// BF16 Gram for large modes (BF16 MFMA v_mfma_f32_16x16x32_bf16, FP32 accumulation within a
// contraction chunk of at most 8192 indices, FP64 across chunks).  128x128 tiles of G, each of the
// four waves owning a 64x64 quarter (sixteen 16x16 accumulators), 64 contraction indices per
// stage.  Staging moves 16-byte vectors: along the contraction index for modes 1 and 2 (written to
// LDS as they are), along the row index for mode 3 (written transposed, eight 2-byte stores); the
// loaded vectors stay raw in registers through the previous stage's MFMAs and are masked only at
// the LDS store.  Fragment layout: lane (i, q) holds elements 8q .. 8q + 7 of row i of a 16-row
// block (both operands the same way, so each instruction pairs matching contraction indices).
constexpr int GB_T = 128;
constexpr int GB_NT = 256;
constexpr int GB_KC = 128;                       // a stage's MFMAs cover the next stage's loads
constexpr int GB_LD = GB_KC + 8;                        // LDS row pitch in bf16 elements
constexpr int GB_VPT = GB_T * GB_KC / 8 / GB_NT;        // 16-byte vectors per thread and operand
constexpr int GB_MAXCHUNK = 8192;

typedef unsigned int gb_u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 gb_bf16x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(GB_NT) void gram_bf16_big_kernel(const uint16_t* __restrict__ src, GramGeom g,
                                                              double* __restrict__ part) {
  __shared__ __align__(16) uint16_t Xm[GB_T][GB_LD];
  __shared__ __align__(16) uint16_t Xn[GB_T][GB_LD];
  const int L = blockIdx.x;
  const int xcd = L & 7, idx = L >> 3;
  const int tile = idx % g.nupper;
  const int split = (idx / g.nupper) * 8 + xcd;
  if (split >= g.nsplit) return;
  int tm, tn;
  tile_of(tile, g.ntile, tm, tn);
  const bool diag = (tm == tn);
  const int kbeg = split * g.kchunk, kend = min(g.Ktot, kbeg + g.kchunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, i = lane & 15, q = lane >> 4;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  const bool v0 = g.variant == 0;
  const int gM = g.M, gK = g.K, sm = g.sm, sk = g.sk;
  const long long sb = g.sb;
  const double invK = 1.0 / (double)(v0 ? gK : 1);
  // vector v of this thread: variant 0 -> (row, 8 contraction indices); variant 1 -> (8 rows, one
  // index), the thread's GB_VPT vectors at consecutive indices of the same 8 rows so that they are
  // written to LDS as one 8-byte word per row
  static_assert(GB_VPT == 8 && GB_KC == GB_VPT * (GB_NT / (GB_T / 8)), "variant-1 staging covers the stage");
  auto vrow = [=](int v) {
    const int e = tid + v * GB_NT;
    return v0 ? e / (GB_KC / 8) : (tid % (GB_T / 8)) * 8;
  };
  auto vk = [=](int v) {
    const int e = tid + v * GB_NT;
    return v0 ? (e % (GB_KC / 8)) * 8 : GB_VPT * (tid / (GB_T / 8)) + v;
  };
  auto addr = [=](int m, int kp) -> long long {
    if (v0) {
      const int b = (int)(((double)kp + 0.5) * invK);
      return (long long)b * sb + (long long)m * sm + (kp - b * gK);
    }
    return (long long)kp * sk + m;
  };
  gb_u32x4 rm[GB_VPT], rn[GB_VPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int v = 0; v < GB_VPT; ++v) {
      const int r = vrow(v), kp = k0 + vk(v);
      const bool okk = kp < kend;
      const int gm = tm * GB_T + r, gn = tn * GB_T + r;
      rm[v] = *(const gb_u32x4*)(src + addr(gm < gM && okk ? gm : 0, okk ? kp : 0));
      if (!diag) rn[v] = *(const gb_u32x4*)(src + addr(gn < gM && okk ? gn : 0, okk ? kp : 0));
    }
  };
  auto put = [&](uint16_t (*X)[GB_LD], const gb_u32x4* raw, int row0, int k0) {
    if (v0) {
#pragma unroll
      for (int v = 0; v < GB_VPT; ++v) {
        const int r = vrow(v), kk = vk(v);
        const bool ok = row0 + r < gM && k0 + kk < kend;   // whole vectors are in or out of range
        *(gb_u32x4*)&X[r][kk] = ok ? raw[v] : gb_u32x4{0u, 0u, 0u, 0u};
      }
    } else {
      // eight vectors = rows r .. r+7 at indices kk .. kk+7: row r + e gets the 16-byte word
      // (element e of vectors 0..7)
      const int r = vrow(0), kk = vk(0);
      gb_u32x4 val[GB_VPT];
#pragma unroll
      for (int v = 0; v < GB_VPT; ++v) {
        const bool ok = row0 + r < gM && k0 + kk + v < kend;
        val[v] = ok ? raw[v] : gb_u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int sh = 16 * (e & 1);
        uint32_t h[GB_VPT];
#pragma unroll
        for (int v = 0; v < GB_VPT; ++v) h[v] = (val[v][e >> 1] >> sh) & 0xFFFFu;
        *(gb_u32x4*)&X[r + e][kk] = gb_u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                            h[6] | (h[7] << 16)};
      }
    }
  };
  flt4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
  uint16_t (*Bn)[GB_LD] = diag ? Xm : Xn;
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GB_KC) {
    put(Xm, rm, tm * GB_T, k0);
    if (!diag) put(Xn, rn, tn * GB_T, k0);
    __syncthreads();
    if (k0 + GB_KC < kend) fetch(k0 + GB_KC);
#pragma unroll
    for (int ks = 0; ks < GB_KC; ks += 32) {
      gb_u32x4 fa[4], fb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = *(const gb_u32x4*)&Xm[wm + 16 * a + i][ks + 8 * q];
#pragma unroll
      for (int b = 0; b < 4; ++b) fb[b] = *(const gb_u32x4*)&Bn[wn + 16 * b + i][ks + 8 * q];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(gb_bf16x8, fa[a]),
                                                              __builtin_bit_cast(gb_bf16x8, fb[b]), acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[4 q + v][i] of a 16x16 block is element v of lane i + 16 q
  double* out = part + ((long long)tile * g.nsplit + split) * (GB_T * GB_T);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(wm + 16 * a + 4 * q + v) * GB_T + wn + 16 * b + i] = (double)acc[a][b][v];
}

// FP64 Gram for large modes from FP64 or FP32 input: 128x128 tiles of G, each of the four waves a
// 64x64 quarter (sixteen 16x16 accumulators on v_mfma_f64_16x16x4f64); on diagonal tiles the 16x16
// blocks below the diagonal are skipped (the reduction reads the upper triangle only) and the
// quarter below the diagonal takes the lower half of the off-diagonal quarter's rows (10, 8, 8 and
// 10 blocks instead of 10, 0, 16 and 10); blocks past the last row are skipped everywhere.
constexpr int GF_T = 128;
constexpr int GF_NT = 256;
constexpr int GF_KC = 16;   // contraction indices per stage

// The operands go straight from memory into registers: no LDS and no barrier.  The contraction is
// a sum, so any order of its indices that both operands share gives the same products: within a
// stage of 16 indices, lane (p, q) of a 16x4 fragment holds index k0 + 4q + e at MFMA step e for
// modes 1 and 2 (one 16-byte load of four consecutive indices per row block), and index
// k0 + 4e + q for mode 3, whose unfolding is contiguous along the row (one element per row block
// and step).  Each wave loads its own rows (its partner wave's copy of the same rows comes from the
// cache), keeps the next stage's loads in flight in a second register set while the current one
// is multiplied, and promotes to FP64 just before the MFMAs.  Full stages run without masks; the
// chunk's last partial stage zeroes the indices past its end.
// PAT: the wave's 16x16 blocks (bit 4i + j) fixed at compile time, or 0 for the runtime mask `on`
template <class T, unsigned PAT>
__device__ __forceinline__ void gd_stage(dbl4 (&acc)[4][4], const T (&ra)[4][4], const T (&rb)[4][4],
                                         const bool (&on)[4][4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = (double)ra[i][e];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = (double)rb[j][e];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (PAT ? ((PAT >> (4 * i + j)) & 1u) != 0 : on[i][j])
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

template <class T, int VAR, unsigned PAT>
__device__ __forceinline__ void gd_chunk(const T* __restrict__ src, const GramGeom& g, const int (&gra)[4],
                                         const int (&grb)[4], int kbeg, int kend, dbl4 (&acc)[4][4],
                                         const bool (&on)[4][4]) {
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  const int lane = threadIdx.x & 63, q = lane >> 4;
  constexpr bool v0 = VAR == 0;
  const double invK = 1.0 / (double)(v0 ? g.K : 1);
  const int kmaxv = g.Ktot - VW, kmax1 = g.Ktot - 1;
  // one operand's stage at k0 into r; `mask` zeroes indices >= kend (the chunk's last stage only)
  auto load = [&](T (&r)[4][4], const int (&gr)[4], int k0, bool mask) {
    if constexpr (v0) {
#pragma unroll
      for (int u = 0; u < 4 / VW; ++u) {
        const int kk = k0 + 4 * q + u * VW;
        const int ks = min(kk, kmaxv);
        const int b = (int)(((double)ks + 0.5) * invK);
        const long long off = (long long)b * g.sb + (ks - b * g.K);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const vec_t v = *(const vec_t*)(src + off + (long long)gr[i] * g.sm);
#pragma unroll
          for (int t = 0; t < VW; ++t) r[i][u * VW + t] = (mask && kk + t >= kend) ? (T)0 : v[t];
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = k0 + 4 * e + q;
        const long long off = (long long)min(kk, kmax1) * g.sk;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T v = src[off + gr[i]];
          r[i][e] = (mask && kk >= kend) ? (T)0 : v;
        }
      }
    }
  };
  T ra0[4][4], rb0[4][4], ra1[4][4], rb1[4][4];
  const int nst = (kend - kbeg) / GF_KC, kfull = kbeg + GF_KC * nst;
  if (nst > 0) {
    load(ra0, gra, kbeg, false);
    load(rb0, grb, kbeg, false);
  }
  int s = 0;
  for (; s + 2 <= nst; s += 2) {
    const int k0 = kbeg + GF_KC * s;
    load(ra1, gra, k0 + GF_KC, false);
    load(rb1, grb, k0 + GF_KC, false);
    __builtin_amdgcn_sched_barrier(0);
    gd_stage<T, PAT>(acc, ra0, rb0, on);
    __builtin_amdgcn_sched_barrier(0);
    // stage s + 2 (clamped indices and unused when the chunk ends at s + 2)
    load(ra0, gra, k0 + 2 * GF_KC, false);
    load(rb0, grb, k0 + 2 * GF_KC, false);
    __builtin_amdgcn_sched_barrier(0);
    gd_stage<T, PAT>(acc, ra1, rb1, on);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (s < nst) gd_stage<T, PAT>(acc, ra0, rb0, on);
  if (kfull < kend) {
    load(ra1, gra, kfull, true);
    load(rb1, grb, kfull, true);
    gd_stage<T, PAT>(acc, ra1, rb1, on);
  }
}

// FP32 input fits two waves per SIMD (240 registers); FP64 input's stages take one.
template <class T, int VAR>
__global__ __launch_bounds__(GF_NT, sizeof(T) == 4 ? 2 : 1) void gram_f64_direct_kernel(
    const T* __restrict__ src, GramGeom g, double* __restrict__ part) {
  const int L = blockIdx.x;
  const int xcd = L & 7, idx = L >> 3;
  // launch order: every off-diagonal tile's workgroups first, then the diagonal tiles' (at most 10
  // of 16 blocks per wave), so that the last round, which runs ragged, holds the shorter ones
  // (600^3: 2.52 against 2.58 ms per mode); within each class consecutive workgroups of one XCD
  // take the tiles of one split, whose rows they then share in that XCD's L2
  const int nd = g.ntile, no = g.nupper - nd, per = g.nsplit / 8;
  int tm, tn, split;
  if (idx < no * per) {
    const int to = idx % no;
    split = (idx / no) * 8 + xcd;
    int row = 0, start = 0;   // the to-th off-diagonal tile of the upper triangle, row by row
    while (to >= start + (g.ntile - 1 - row)) { start += g.ntile - 1 - row; ++row; }
    tm = row;
    tn = row + 1 + (to - start);
  } else {
    const int id = idx - no * per;
    tm = tn = id % nd;
    split = (id / nd) * 8 + xcd;
  }
  if (split >= g.nsplit) return;
  const int tile = tm * g.ntile - tm * (tm - 1) / 2 + (tn - tm);
  const bool diag = (tm == tn);
  const int kbeg = split * g.kchunk, kend = min(g.Ktot, kbeg + g.kchunk);
  // the wave index as a wave-uniform value: the quarter's geometry stays in scalar registers
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // wave quarters (diagonal tiles: 10, 8, 8 and 10 blocks)
  int wm = (w & 1) * 64, wn = (w >> 1) * 64, ilim = 4;
  if (diag && w == 1) { wm = 32; wn = 64; ilim = 2; }
  if (diag && w == 2) ilim = 2;
  bool on[4][4];
  unsigned mask = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r0 = wm + 16 * i, c0 = wn + 16 * j;
      on[i][j] = i < ilim && tm * GF_T + r0 < g.M && tn * GF_T + c0 < g.M && (!diag || r0 <= c0);
      mask |= on[i][j] ? 1u << (4 * i + j) : 0u;
    }
  // nothing inside the matrix: no loads, no partial entries the reduction reads
  if (mask == 0) return;
  // rows of this lane in each row block (clamped into the matrix: rows past the end only feed
  // partial entries that the reduction never reads)
  int gra[4], grb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gra[i] = min(tm * GF_T + wm + 16 * i + (lane & 15), g.M - 1);
    grb[i] = min(tn * GF_T + wn + 16 * i + (lane & 15), g.M - 1);
  }
  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  // the block patterns of whole quarters, upper triangles of diagonal quarters and the two-row
  // and two-column quarters at the edges run without per-MFMA masks (and without the loads of
  // operand blocks they do not use)
  switch (mask) {
    case 0xffffu: gd_chunk<T, VAR, 0xffffu>(src, g, gra, grb, kbeg, kend, acc, on); break;
    case 0x8cefu: gd_chunk<T, VAR, 0x8cefu>(src, g, gra, grb, kbeg, kend, acc, on); break;
    case 0x00ffu: gd_chunk<T, VAR, 0x00ffu>(src, g, gra, grb, kbeg, kend, acc, on); break;
    case 0x3333u: gd_chunk<T, VAR, 0x3333u>(src, g, gra, grb, kbeg, kend, acc, on); break;
    default: gd_chunk<T, VAR, 0u>(src, g, gra, grb, kbeg, kend, acc, on); break;
  }
  double* out = part + ((long long)tile * g.nsplit + split) * (GF_T * GF_T);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i < ilim)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = wm + 16 * i + 4 * v + (lane >> 4);
          const int c = wn + 16 * j + (lane & 15);
          out[r * GF_T + c] = acc[i][j][v];
        }
}

GramGeom make_geom_base(const int64_t dims[3], int mode) {
  GramGeom g{};
  const long long I1 = dims[0], I2 = dims[1], I3 = dims[2];
  if (mode == 0) {
    g.variant = 0; g.M = (int)I1; g.K = (int)(I2 * I3); g.Ktot = g.K; g.sb = 0; g.sm = (int)(I2 * I3);
  } else if (mode == 1) {
    g.variant = 0; g.M = (int)I2; g.K = (int)I3; g.Ktot = (int)(I1 * I3); g.sb = I2 * I3; g.sm = (int)I3;
  } else {
    g.variant = 1; g.M = (int)I3; g.Ktot = (int)(I1 * I2); g.sk = (int)I3;
  }
  return g;
}

// Small Grams (M <= 208), FP64 path: one workgroup per split-K chunk computes every upper-triangle
// 16x16 tile of G from its chunk, which it holds for all M rows in LDS.  Each tensor element is
// read once, and the partials are one triangle per chunk (at M = 200: 91 tiles, 47 MB for 250
// chunks) instead of one 64x64 tile per (tile, chunk) pair (105 MB), with 64x64 tiles that are
// 22 % padding at M = 200.  Twelve waves take the tiles round robin.
constexpr int GT_NW = 12;
constexpr int GT_NT = 64 * GT_NW;
constexpr int GT_KC = 32;            // contraction indices per stage
constexpr int GT_LD = GT_KC + 1;     // LDS row pitch (doubles)
constexpr int GT_MAXM = 208;   // up to 91 tiles, 8 per wave: accumulators stay in registers
constexpr int GT_PER = (GT_MAXM * GT_KC + GT_NT - 1) / GT_NT;   // staged elements per thread and stage

template <class T, int NTW>
__global__ __launch_bounds__(GT_NT) void gram_tri_kernel(const T* __restrict__ src, GramGeom g, int mp,
                                                         double* __restrict__ part) {
  extern __shared__ double xs[];   // [mp][GT_LD]
  const int nt = mp / 16, ntri = nt * (nt + 1) / 2;
  const int split = blockIdx.x;
  const int kbeg = split * g.kchunk, kend = min(g.Ktot, kbeg + g.kchunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  const double invK = 1.0 / (double)(g.variant == 0 ? g.K : 1);
  int ti[NTW], tj[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    // (row, column) of upper-triangle tile t, rows enumerated in order; a fixed-trip search so the
    // surrounding loop unrolls and ti / tj stay in registers
    const int t = w + GT_NW * j < ntri ? w + GT_NW * j : 0;
    int row = 0, start = 0;
#pragma unroll
    for (int rr = 0; rr < GT_MAXM / 16; ++rr) {
      const bool next = rr == row && rr < nt && t >= start + (nt - rr);
      start += next ? nt - rr : 0;
      row += next ? 1 : 0;
    }
    ti[j] = row;
    tj[j] = row + (t - start);
  }
  dbl4 acc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
  // staging slot s of this thread: element e = tid + s GT_NT of the mp x GT_KC stage, along the
  // index that is contiguous in memory (k for variant 0, the row for variant 1)
  const int nel = mp * GT_KC;
  T rv[GT_PER];   // raw staged values: masked and converted only when written to LDS, so the
                  // loads stay in flight through the previous stage's MFMAs
  const bool rowk = g.variant == 0;
  auto slot = [=](int s) {   // (row, k) of slot s, returned by value
    const int e = tid + s * GT_NT;
    const int m0 = e / GT_KC, k0 = e & (GT_KC - 1), k1 = e / mp, m1 = e - k1 * mp;
    return rowk ? int2{m0, k0} : int2{m1, k1};
  };
  // element (m, kp) of the unfolding, from scalar strides (variant 0 splits kp = b K + k by a
  // double-precision reciprocal, exact for kp < 2^26)
  const bool v0 = g.variant == 0;
  const int gM = g.M, gK = g.K, sm = g.sm, sk = g.sk;
  const long long sb = g.sb;
  auto addr = [=](int m, int kp) -> long long {
    if (v0) {
      const int b = (int)(((double)kp + 0.5) * invK);
      return (long long)b * sb + (long long)m * sm + (kp - b * gK);
    }
    return (long long)kp * sk + m;
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < GT_PER; ++s) {
      const int2 mk = slot(s);
      const int m = mk.x, kk = mk.y;
      const int kp = k0 + kk;
      const bool ok = tid + s * GT_NT < nel && m < gM && kp < kend;
      rv[s] = src[addr(ok ? m : 0, ok ? kp : 0)];
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GT_KC) {
#pragma unroll
    for (int s = 0; s < GT_PER; ++s) {
      const int2 mk = slot(s);
      const bool ok = mk.x < gM && k0 + mk.y < kend;
      if (tid + s * GT_NT < nel) xs[mk.x * GT_LD + mk.y] = ok ? conv<double, T>(rv[s]) : 0.0;
    }
    __syncthreads();
    if (k0 + GT_KC < kend) fetch(k0 + GT_KC);
#pragma unroll
    for (int kk = 0; kk < GT_KC; kk += 4) {
      // every slot runs (a slot past the last tile repeats tile 0 and is not written): no branch,
      // so the LDS reads of a k-step are issued together ahead of its MFMAs.
      // A fragment: lane holds A[lane%16][lane/16]; B fragment: B[lane/16][lane%16]
      double a[NTW], b[NTW];
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        a[j] = xs[(16 * ti[j] + r) * GT_LD + kk + q];
        b[j] = xs[(16 * tj[j] + r) * GT_LD + kk + q];
      }
#pragma unroll
      for (int j = 0; j < NTW; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[j], acc[j], 0, 0, 0);
      // keep the next k-step's reads below this point: hoisted further they would need more
      // registers than the accumulators leave
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
  // D[4 v + lane/16][lane%16] is acc[v] (result layout of v_mfma_f64_16x16x4f64)
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int t = w + GT_NW * j;
    if (t < ntri) {
      double* out = part + ((long long)split * ntri + t) * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(4 * v + q) * 16 + r] = acc[j][v];
    }
  }
}

// G[m][n] = G[n][m] = sum over chunks of the partial triangles: 32 entries per 256-thread block,
// eight threads per entry each adding every eighth chunk (four interleaved sums, so loads stay in
// flight), the eight results combined in a fixed order (bit-reproducible).
__global__ __launch_bounds__(256) void gram_tri_reduce_kernel(const double* __restrict__ part, int M, int mp,
                                                              int nsplit, double* __restrict__ G) {
  __shared__ double red[8][33];
  const int nt = mp / 16, ntri = nt * (nt + 1) / 2;
  const int o = threadIdx.x & 31, qq = threadIdx.x >> 5;
  const long long n = (long long)ntri * 256;
  const long long e = (long long)blockIdx.x * 32 + o;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < n) {
    int sp = qq;
    for (; sp + 24 < nsplit; sp += 32) {
      s0 += part[(long long)sp * n + e];
      s1 += part[(long long)(sp + 8) * n + e];
      s2 += part[(long long)(sp + 16) * n + e];
      s3 += part[(long long)(sp + 24) * n + e];
    }
    for (; sp < nsplit; sp += 8) s0 += part[(long long)sp * n + e];
  }
  red[qq][o] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (qq == 0 && e < n) {
    const int t = (int)(e >> 8), rc = (int)(e & 255), rr = rc >> 4, cc = rc & 15;
    int tm, tn;
    tile_of(t, nt, tm, tn);
    const int m = tm * 16 + rr, c = tn * 16 + cc;
    if ((tm != tn || rr <= cc) && m < M && c < M) {
      const double v = ((red[0][o] + red[1][o]) + (red[2][o] + red[3][o])) +
                       ((red[4][o] + red[5][o]) + (red[6][o] + red[7][o]));
      G[(long long)m * M + c] = v;
      G[(long long)c * M + m] = v;
    }
  }
}

// Split of the contraction for gram_tri_kernel: about 256 chunks (one workgroup per CU), each a
// multiple of the stage length.
GramGeom make_tri_geom(const int64_t dims[3], int mode, int* mp) {
  GramGeom g = make_geom_base(dims, mode);
  *mp = (g.M + 15) / 16 * 16;
  long long chunk = (g.Ktot + 255) / 256;
  chunk = (chunk + GT_KC - 1) / GT_KC * GT_KC;
  g.kchunk = (int)chunk;
  g.nsplit = (int)((g.Ktot + chunk - 1) / chunk);
  return g;
}

GramGeom make_geom(const int64_t dims[3], int mode, int bk) {
  GramGeom g = make_geom_base(dims, mode);
  g.ntile = (g.M + TILE - 1) / TILE;
  g.nupper = g.ntile * (g.ntile + 1) / 2;
  // aim for ~4096 workgroups (16 per CU: more waves in flight hide the staging latency; measured
  // 17 % faster than 1024 at 200^3) without chunks shorter than 4 k-tiles
  long long want = (4096 + g.nupper - 1) / g.nupper;
  long long maxsplit = (g.Ktot + 4 * bk - 1) / (4 * bk);
  long long ns = want < maxsplit ? want : maxsplit;
  if (ns < 1) ns = 1;
  ns = (ns + 7) / 8 * 8;
  long long chunk = (g.Ktot + ns - 1) / ns;
  chunk = (chunk + bk - 1) / bk * bk;
  ns = (g.Ktot + chunk - 1) / chunk;
  ns = (ns + 7) / 8 * 8;
  g.nsplit = (int)ns;
  g.kchunk = (int)chunk;
  return g;
}

bool use_bf16(int dtype, int compute_dtype) { return dtype == CPD_BF16 && compute_dtype == CPD_BF16; }

// 128x128 tiles for the large BF16 Gram: chunks of at most GB_MAXCHUNK indices (a multiple of the
// stage), split count a multiple of 8 (XCD order) and at least ~512 workgroups.
GramGeom make_big_geom(const int64_t dims[3], int mode) {
  GramGeom g = make_geom_base(dims, mode);
  g.ntile = (g.M + GB_T - 1) / GB_T;
  g.nupper = g.ntile * (g.ntile + 1) / 2;
  long long ns = (512 + g.nupper - 1) / g.nupper;
  const long long minsplit = (g.Ktot + GB_MAXCHUNK - 1) / GB_MAXCHUNK;
  if (ns < minsplit) ns = minsplit;
  ns = (ns + 7) / 8 * 8;
  long long chunk = (g.Ktot + ns - 1) / ns;
  chunk = (chunk + GB_KC - 1) / GB_KC * GB_KC;
  ns = (g.Ktot + chunk - 1) / chunk;
  ns = (ns + 7) / 8 * 8;
  g.nsplit = (int)ns;
  g.kchunk = (int)chunk;
  return g;
}

// 128x128 FP64 tiles: the split count is a multiple of 8 (XCD order), chunks hold at least 32
// stages, and the workgroup count fills GF_SLOTS resident workgroups (two per compute unit on the
// 256 units) in whole rounds: the first count of at least eight rounds within 2 % of full, else the
// fullest one seen.  Diagonal tiles finish early and the last round is ragged, so more, shorter
// rounds pay for the larger partials (600^3: 272 splits, 2.53 ms per mode against 2.61 ms with 136).
constexpr int GF_SLOTS = 512;

GramGeom make_f64_big_geom(const int64_t dims[3], int mode) {
  GramGeom g = make_geom_base(dims, mode);
  g.ntile = (g.M + GF_T - 1) / GF_T;
  g.nupper = g.ntile * (g.ntile + 1) / 2;
  const long long maxsplit = (g.Ktot + 32 * GF_KC - 1) / (32 * GF_KC);
  long long best_ns = 8, best_chunk = (g.Ktot + 7) / 8;
  best_chunk = (best_chunk + GF_KC - 1) / GF_KC * GF_KC;
  double best_eff = -1.0;
  for (long long want = 8; want <= 1024; want += 8) {
    long long chunk = (g.Ktot + want - 1) / want;
    chunk = (chunk + GF_KC - 1) / GF_KC * GF_KC;
    long long ns = (g.Ktot + chunk - 1) / chunk;
    ns = (ns + 7) / 8 * 8;
    const long long n = (long long)g.nupper * ns;
    const long long rounds = (n + GF_SLOTS - 1) / GF_SLOTS;
    const double eff = (double)n / (double)(rounds * GF_SLOTS);
    if (eff > best_eff + 1e-12) {
      best_eff = eff;
      best_ns = ns;
      best_chunk = chunk;
    }
    if (rounds >= 8 && eff >= 0.98) {
      best_ns = ns;
      best_chunk = chunk;
      break;
    }
    if (want >= maxsplit) break;
  }
  g.nsplit = (int)best_ns;
  g.kchunk = (int)best_chunk;
  return g;
}

// The 128x128 FP64 kernel moves whole 16-byte vectors of the input type.
bool big_f64_ok(const GramGeom& g, const void* T, int dtype) {
  if ((dtype != CPD_F64 && dtype != CPD_F32) || g.M <= GT_MAXM || ((uintptr_t)T & 15)) return false;
  const int vw = dtype == CPD_F64 ? 2 : 4;
  if (g.variant == 0) return g.K % vw == 0 && g.sm % vw == 0 && g.sb % vw == 0;
  return g.sk % vw == 0 && g.M % vw == 0;
}

// The large BF16 kernel moves whole 16-byte vectors: every vector must be in one slab and aligned.
bool big_bf16_ok(const GramGeom& g, const void* T) {
  if (g.M <= GT_MAXM || ((uintptr_t)T & 15)) return false;
  if (g.variant == 0) return g.K % 8 == 0 && g.sm % 8 == 0 && g.sb % 8 == 0;
  return g.sk % 8 == 0 && g.M % 8 == 0;
}

template <class T>
cpd_status launch_tri(const void* src, const GramGeom& g, int mp, int ntw, size_t lds, double* part, hipStream_t s) {
  const dim3 grid(g.nsplit), block(GT_NT);
  const T* p = (const T*)src;
  auto k = ntw <= 1 ? gram_tri_kernel<T, 1> : ntw <= 3 ? gram_tri_kernel<T, 3> : gram_tri_kernel<T, 8>;
  if (lds > 64 * 1024)
    CPD_HIP_CHECK(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, grid, block, lds, s, p, g, mp, part);
  return CPD_OK;
}

}  // namespace

size_t gram_ws_bytes(const int64_t dims[3], int mode) {
  const GramGeom g = make_geom(dims, mode, BK), h = make_geom(dims, mode, BKH);
  const int ns = g.nsplit > h.nsplit ? g.nsplit : h.nsplit;
  size_t b = align_up((size_t)g.nupper * ns * TILE * TILE * sizeof(double), 256);
  if (g.M > GT_MAXM) {
    const GramGeom gb = make_big_geom(dims, mode);
    const size_t bb = align_up((size_t)gb.nupper * gb.nsplit * GB_T * GB_T * sizeof(double), 256);
    b = b > bb ? b : bb;
    const GramGeom gf = make_f64_big_geom(dims, mode);
    const size_t bf = align_up((size_t)gf.nupper * gf.nsplit * GF_T * GF_T * sizeof(double), 256);
    b = b > bf ? b : bf;
  }
  if (g.M <= GT_MAXM) {
    int mp;
    const GramGeom t = make_tri_geom(dims, mode, &mp);
    const size_t nt = mp / 16;
    const size_t bt = align_up((size_t)t.nsplit * (nt * (nt + 1) / 2) * 256 * sizeof(double), 256);
    b = b > bt ? b : bt;
  }
  return b;
}

cpd_status gram(const void* T, int dtype, const int64_t dims[3], int mode, int compute_dtype,
                double* G, void* ws, size_t ws_bytes, hipStream_t s) {
  if (mode < 0 || mode > 2 || T == nullptr || G == nullptr) {
    set_error("gram: bad arguments");
    return CPD_E_INVALID;
  }
  const bool bf = use_bf16(dtype, compute_dtype);
  GramGeom g = make_geom(dims, mode, bf ? BKH : BK);
  const size_t need = gram_ws_bytes(dims, mode);
  if (ws == nullptr || ws_bytes < need) {
    set_error("gram: workspace %zu < %zu", ws_bytes, need);
    return CPD_E_WORKSPACE;
  }
  double* part = (double*)ws;
  if (!bf && g.M <= GT_MAXM) {
    int mp;
    const GramGeom t = make_tri_geom(dims, mode, &mp);
    const int nt = mp / 16, ntri = nt * (nt + 1) / 2;
    const int ntw = (ntri + GT_NW - 1) / GT_NW;
    const size_t lds = (size_t)mp * GT_LD * sizeof(double);
    prof_begin(CPD_PK_GRAM, s);
    cpd_status st = CPD_OK;
    switch (dtype) {
      case CPD_F64: st = launch_tri<double>(T, t, mp, ntw, lds, part, s); break;
      case CPD_F32: st = launch_tri<float>(T, t, mp, ntw, lds, part, s); break;
      case CPD_BF16: st = launch_tri<uint16_t>(T, t, mp, ntw, lds, part, s); break;
      default: set_error("gram: bad dtype %d", dtype); return CPD_E_INVALID;
    }
    if (st) return st;
    const long long nel = (long long)ntri * 256;
    hipLaunchKernelGGL(gram_tri_reduce_kernel, dim3((unsigned)((nel + 31) / 32)), dim3(256), 0, s, part, t.M, mp,
                       t.nsplit, G);
    prof_end(CPD_PK_GRAM, s);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  if (!bf && big_f64_ok(make_geom_base(dims, mode), T, dtype)) {
    const GramGeom gf = make_f64_big_geom(dims, mode);
    const int nb = gf.nupper * gf.nsplit;
    prof_begin(CPD_PK_GRAM, s);
    auto k = dtype == CPD_F64 ? (gf.variant == 0 ? (const void*)gram_f64_direct_kernel<double, 0>
                                                 : (const void*)gram_f64_direct_kernel<double, 1>)
                              : (gf.variant == 0 ? (const void*)gram_f64_direct_kernel<float, 0>
                                                 : (const void*)gram_f64_direct_kernel<float, 1>);
    void* args[] = {(void*)&T, (void*)&gf, (void*)&part};
    CPD_HIP_CHECK(hipLaunchKernel(k, dim3(nb), dim3(GF_NT), args, 0, s));
    CPD_LAUNCH_CHECK();
    const long long nelf = (long long)gf.nupper * GF_T * GF_T;
    hipLaunchKernelGGL(gram_reduce_kernel<GF_T>, dim3((unsigned)((nelf + 255) / 256)), dim3(256), 0, s, part, gf, G);
    prof_end(CPD_PK_GRAM, s);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  if (bf && big_bf16_ok(make_geom_base(dims, mode), T)) {
    const GramGeom gb = make_big_geom(dims, mode);
    prof_begin(CPD_PK_GRAM, s);
    hipLaunchKernelGGL(gram_bf16_big_kernel, dim3(gb.nupper * gb.nsplit), dim3(GB_NT), 0, s, (const uint16_t*)T, gb,
                       part);
    CPD_LAUNCH_CHECK();
    const long long nelb = (long long)gb.nupper * GB_T * GB_T;
    hipLaunchKernelGGL(gram_reduce_kernel<GB_T>, dim3((unsigned)((nelb + 255) / 256)), dim3(256), 0, s, part, gb, G);
    prof_end(CPD_PK_GRAM, s);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
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
      if (bf)
        hipLaunchKernelGGL(gram_partial_bf16_kernel, dim3(nblocks), dim3(NT), 0, s, (const uint16_t*)T, g, part);
      else
        hipLaunchKernelGGL(gram_partial_kernel<uint16_t>, dim3(nblocks), dim3(NT), 0, s, (const uint16_t*)T, g, part);
      break;
    default:
      set_error("gram: bad dtype %d", dtype);
      return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  const long long nel = (long long)g.nupper * TILE * TILE;
  hipLaunchKernelGGL(gram_reduce_kernel<TILE>, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s,
                     part, g, G);
  prof_end(CPD_PK_GRAM, s);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
