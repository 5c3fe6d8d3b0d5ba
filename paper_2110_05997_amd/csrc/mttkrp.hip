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
// FP32- and BF16-matrix-core variants (FP32 accumulation) of the same contraction follow the FP64
// kernel; they differ in data flow, see the comment above mttkrp_lp_kernel.
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

// ---------------------------------------------------------------------------------------------
// FP32 / BF16 matrix-core MTTKRP, FP32 accumulation.  M[m][r] = sum_x Wa[x][r] sum_y T[m, x, y]
// Wb[y][r] as in the FP64 kernel, with a data flow built for a contraction that is bound by HBM
// (BF16) or by the FP32 matrix rate rather than by the FP64 one:
//  * the inner factor Wb is first copied, rounded to the MFMA input type, into a zero-padded
//    column-major array WbF[col][y] (col < 16 NCT, y < ypad, ypad a multiple of the k-group), so
//    every B fragment is one 16-byte load from a small L1/L2-resident array: no LDS staging and
//    no barrier in the main loop;
//  * each lane loads its own A fragment straight from the tensor: KS = LP_KSUB * KPL consecutive
//    inner indices of one row, as LP_KSUB 16-byte (8-byte for BF16 data on the FP32 cores) vector
//    loads when the inner index is contiguous and aligned (modes 1, 2), else as scalar loads
//    that are coalesced along the contiguous row index (mode 3).  A step covers a k-group of
//    4 KS inner indices, so a row is read in 4 KS-element runs (128 bytes for LP_KSUB = 2): whole
//    cache lines, which HBM serves far better than the half lines of one vector per lane;
//  * sub-vector s of lane (i, q) holds inner indices y0 + 4 KPL s + KPL q + e (e < KPL), so the
//    four lanes of a row read one contiguous 64-byte run per load instruction.  F32:
//    v_mfma_f32_16x16x4f32, element e feeds instruction (s, e); BF16: v_mfma_f32_16x16x32_bf16, the
//    KPL = 8 elements feed instruction s.  A and B use the same lane/element -> inner-index map, so
//    each instruction adds the products of matching indices whatever the hardware's k order;
//  * a wave owns LP_RB 16-row blocks and every WX-th outer index x of its workgroup's range; the
//    inner sum over y of one x (FP32 MFMA accumulator) is scaled by Wa[x] (rounded to FP32) and
//    added into a second FP32 accumulator; the WX wave groups are added through LDS in a fixed
//    order and written as one FP64 partial per workgroup, summed by mttkrp_reduce_kernel.
constexpr int LP_RB = 2;                        // 16-row blocks per wave
constexpr int LP_WR = 2;                        // waves along the rows
constexpr int LP_WX = 4;                        // waves along the outer index
constexpr int LP_DA = 3;                        // steps whose A fragments are in flight per wave
constexpr int LP_KSUB = 2;                      // 16-byte vectors per lane, row and step
constexpr int LP_XMAX = 64;                     // outer indices per workgroup (Wa rows in LDS)
constexpr int LP_ROWS = 16 * LP_RB * LP_WR;     // rows per workgroup
constexpr int LP_NT = 64 * LP_WR * LP_WX;

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND>
struct LpKind;
template <>
struct LpKind<CPD_F32> {     // v_mfma_f32_16x16x4f32: 4 inner indices per lane and k-group
  static constexpr int KPL = 4;
  typedef float WT;
  typedef flt4 AV;
};
template <>
struct LpKind<CPD_BF16> {    // v_mfma_f32_16x16x32_bf16: 8 inner indices per lane and k-group
  static constexpr int KPL = 8;
  typedef uint16_t WT;
  typedef u32x4 AV;
};

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// Correctly rounded (to nearest even) FP64 -> BF16: truncate to FP32 and make the result odd when
// bits were dropped (round to odd keeps the sticky information), then round to nearest even at
// the BF16 position; exact because FP32 carries more than two bits beyond BF16's eight.
__device__ __forceinline__ uint16_t f64_to_bf16_bits(double v) {
  if (v != v) return 0x7FC0;
  const float t = __double2float_rz(v);
  uint32_t b = __float_as_uint(t);
  if ((double)t != v) b |= 1u;
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

template <int KIND>
__global__ __launch_bounds__(256) void mt_wb_prep_kernel(const double* __restrict__ Wb, int Y, int R, int ypad,
                                                         int ncol, typename LpKind<KIND>::WT* __restrict__ WbF) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)ncol * ypad) return;
  const int col = (int)(e / ypad), y = (int)(e % ypad);
  const double v = (col < R && y < Y) ? Wb[(long long)y * R + col] : 0.0;
  if constexpr (KIND == CPD_F32) WbF[e] = (float)v;
  else WbF[e] = f64_to_bf16_bits(v);
}

// LDS of one workgroup (dynamic): the FP32 Wa rows of its outer range (xper x 16 NCT), then a
// region that holds the inner factor (BLDS: rows 0 .. R-1 of WbF and a zero row R, row pitch
// lp_pitch) during the main loop and the cross-wave reduction buffer after it.
template <int KIND>
__host__ __device__ inline int lp_pitch(int ypad) {
  // elements per LDS row: 16 bytes past a multiple of 128, so the 16 rows one B-fragment read
  // touches start in different banks
  return ypad + 16 / (int)sizeof(typename LpKind<KIND>::WT);
}

template <class TT, int KIND, int MODE, int NCT, bool VEC, bool BLDS>
__global__ __launch_bounds__(LP_NT) void mttkrp_lp_kernel(const TT* __restrict__ T, MtGeom g,
                                                          const double* __restrict__ Wa,
                                                          const typename LpKind<KIND>::WT* __restrict__ WbF,
                                                          int ypad, double* __restrict__ part) {
  typedef LpKind<KIND> K;
  typedef typename K::AV AV;
  typedef typename K::WT WT;
  constexpr int KPL = K::KPL, KS = KPL * LP_KSUB, KG = 4 * KS, NC = NCT * 16;
  extern __shared__ float4 lp_lds[];
  float* const wa_l = (float*)lp_lds;                                            // [xper][NC]
  char* const reg2 = (char*)lp_lds + (((size_t)g.xper * NC * sizeof(float) + 15) / 16) * 16;
  WT* const bl = (WT*)reg2;                                                      // [R + 1][pitch]
  float (*const red)[LP_ROWS][NC + 1] = (float (*)[LP_ROWS][NC + 1])reg2;       // [WX - 1][..][..]
  const int pitch = lp_pitch<KIND>(ypad);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w % LP_WR, wx = w / LP_WR;
  const int i = lane & 15, q = lane >> 4;
  const int split = blockIdx.y;
  const int mw = blockIdx.x * LP_ROWS + wr * 16 * LP_RB;   // first row of this wave
  const int xend = min((split + 1) * g.xper, g.X);
  const int Y = g.Y, R = g.R, ngy = (Y + KG - 1) / KG;

  // A fragment of row block blk for outer index x and k-group yg.  Out-of-range indices are
  // clamped to element 0 of their row and not masked: a row m >= rows only feeds output rows that
  // are never written, and an inner index y >= Y meets a zero B entry (WbF is zero-padded).  So no
  // value is selected after its load, and the loads stay in flight until the MFMA needs them.
  auto load_a = [&](AV (*a)[LP_KSUB], int x, int yg) {
#pragma unroll
    for (int blk = 0; blk < LP_RB; ++blk) {
      const int m = mw + 16 * blk + i;
      const int mc = m < g.rows ? m : 0;
#pragma unroll
      for (int sub = 0; sub < LP_KSUB; ++sub) {
        const int yb = yg * KG + 4 * KPL * sub + KPL * q;
        if constexpr (VEC) {
          const TT* p = t_ptr<TT, MODE>(T, g, mc, x, yb < Y ? yb : 0);
          if constexpr (KIND == CPD_BF16) {
            a[blk][sub] = *(const u32x4*)p;
          } else if constexpr (sizeof(TT) == 4) {
            a[blk][sub] = *(const flt4*)p;
          } else {
            const uint2 u = *(const uint2*)p;
            a[blk][sub] = flt4{bf16_bits_to_f32(u.x & 0xFFFFu), bf16_bits_to_f32(u.x >> 16),
                               bf16_bits_to_f32(u.y & 0xFFFFu), bf16_bits_to_f32(u.y >> 16)};
          }
        } else {
          if constexpr (KIND == CPD_BF16) {
            uint32_t h[KPL];
#pragma unroll
            for (int e = 0; e < KPL; ++e) {
              const int y = yb + e;
              h[e] = *(const uint16_t*)t_ptr<TT, MODE>(T, g, mc, x, y < Y ? y : 0);
            }
            a[blk][sub] = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
          } else {
            float f[KPL];
#pragma unroll
            for (int e = 0; e < KPL; ++e) {
              const int y = yb + e;
              const TT* p = t_ptr<TT, MODE>(T, g, mc, x, y < Y ? y : 0);
              if constexpr (sizeof(TT) == 4) f[e] = *(const float*)p;
              else f[e] = bf16_bits_to_f32(*(const uint16_t*)p);
            }
            a[blk][sub] = flt4{f[0], f[1], f[2], f[3]};
          }
        }
      }
    }
  };
  // B fragments of the NCT column tiles for k-group yg
  auto load_b = [&](AV (*b)[LP_KSUB], int yg) {
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int sub = 0; sub < LP_KSUB; ++sub) {
        const int y = yg * KG + 4 * KPL * sub + KPL * q;
        if constexpr (BLDS) {
          const int row = (c * 16 + i) < R ? (c * 16 + i) : R;   // columns >= R read the zero row
          b[c][sub] = *(const AV*)(bl + row * pitch + y);
        } else {
          b[c][sub] = *(const AV*)(WbF + (long long)(c * 16 + i) * ypad + y);
        }
      }
  };

  flt4 acc[LP_RB][NCT], macc[LP_RB][NCT];
#pragma unroll
  for (int blk = 0; blk < LP_RB; ++blk)
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      acc[blk][c] = flt4{0.f, 0.f, 0.f, 0.f};
      macc[blk][c] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  // Wa rows of this workgroup's outer range, FP32, staged once: the fold then waits only for LDS
  const int xb = split * g.xper;
  for (int e = tid; e < (xend - xb) * NC; e += LP_NT) {
    const int xl = e / NC, col = e - xl * NC;
    wa_l[xl * NC + col] = col < R ? (float)Wa[(long long)(xb + xl) * R + col] : 0.f;
  }
  if constexpr (BLDS) {   // rows 0 .. R-1 of WbF in 16-byte pieces, then the zero row
    const int cpr = ypad * (int)sizeof(WT) / 16;   // pieces per row
    for (int e = tid; e < (R + 1) * cpr; e += LP_NT) {
      const int row = e / cpr, pc = e - row * cpr;
      const uint4 v = row < R ? *(const uint4*)(WbF + (long long)row * ypad + pc * (16 / (int)sizeof(WT)))
                              : uint4{0u, 0u, 0u, 0u};
      *(uint4*)(bl + row * pitch + pc * (16 / (int)sizeof(WT))) = v;
    }
  }
  __syncthreads();
  // the wave's steps are (x, yg) for x = x0, x0 + WX, ... < xend and yg = 0 .. ngy - 1.  Ring slot
  // st % LP_DA holds the A and B fragments of step st; the slot is refilled with step st + LP_DA as
  // soon as its MFMAs are issued.  All vector-memory loads of the loop go through the ring, so the
  // in-order load counter never makes a step wait for anything younger than its own fragments.
  const int x0 = xb + wx;
  const int nsteps = (mw < g.rows && x0 < xend) ? ((xend - x0 + LP_WX - 1) / LP_WX) * ngy : 0;
  if (nsteps > 0) {
    AV ra[LP_DA][LP_RB][LP_KSUB], rb[BLDS ? 1 : LP_DA][NCT][LP_KSUB];
    int lx = x0, lyg = 0, cx = x0, cyg = 0;   // next step to load / to compute
    // the fill is unconditional (a slot past the last step reloads step 0, in range and unused)
    // and kept in slot order (scheduling barrier): the loop head waits for the worst case over
    // its entries, and a branch per slot, or slot 0's loads scheduled last, would make it drain
    // every load in flight on each iteration
#pragma unroll
    for (int d = 0; d < LP_DA; ++d) {
      const bool real = d < nsteps;
      load_a(ra[d], real ? lx : x0, real ? lyg : 0);
      if constexpr (!BLDS) load_b(rb[d], real ? lyg : 0);
      if (real && ++lyg == ngy) { lyg = 0; lx += LP_WX; }
      __builtin_amdgcn_sched_barrier(0);
    }
    // one step: MFMAs on the slot's fragments, optional refill with the step LP_DA ahead, fold
    auto step = [&](AV (&a)[LP_RB][LP_KSUB], AV (&b)[NCT][LP_KSUB], bool refill) {
      if constexpr (BLDS) load_b(b, cyg);   // B from LDS for this step's k-group
      if constexpr (KIND == CPD_BF16) {
#pragma unroll
        for (int sub = 0; sub < LP_KSUB; ++sub)
#pragma unroll
          for (int blk = 0; blk < LP_RB; ++blk)
#pragma unroll
            for (int c = 0; c < NCT; ++c)
              acc[blk][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[blk][sub]),
                                                                    __builtin_bit_cast(bf16x8, b[c][sub]), acc[blk][c],
                                                                    0, 0, 0);
      } else {
#pragma unroll
        for (int sub = 0; sub < LP_KSUB; ++sub)
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int blk = 0; blk < LP_RB; ++blk)
#pragma unroll
              for (int c = 0; c < NCT; ++c)
                acc[blk][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[blk][sub][j], b[c][sub][j], acc[blk][c], 0, 0, 0);
      }
      if (refill) {
        load_a(a, lx, lyg);
        if constexpr (!BLDS) load_b(b, lyg);
        if (++lyg == ngy) { lyg = 0; lx += LP_WX; }
      }
      if (++cyg == ngy) {   // inner sum of cx complete: scale by Wa[cx] and fold
        cyg = 0;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          const float f = wa_l[(cx - xb) * NC + c * 16 + i];
#pragma unroll
          for (int blk = 0; blk < LP_RB; ++blk) {
#pragma unroll
            for (int v = 0; v < 4; ++v) macc[blk][c][v] = fmaf(f, acc[blk][c][v], macc[blk][c][v]);
            acc[blk][c] = flt4{0.f, 0.f, 0.f, 0.f};
          }
        }
        cx += LP_WX;
      }
    };
    // steady state: every refill unconditional (no branch joins for the wait-count bookkeeping)
    int st = 0;
    for (; st + 2 * LP_DA <= nsteps; st += LP_DA) {
#pragma unroll
      for (int d = 0; d < LP_DA; ++d) step(ra[d], rb[BLDS ? 0 : d], true);
    }
    // the last (fewer than 2 LP_DA) steps
#pragma unroll
    for (int d = 0; d < LP_DA; ++d)
      if (st + d < nsteps) step(ra[d], rb[BLDS ? 0 : d], st + d + LP_DA < nsteps);
#pragma unroll
    for (int d = 0; d < LP_DA; ++d)
      if (st + LP_DA + d < nsteps) step(ra[d], rb[BLDS ? 0 : d], false);
  }
  __syncthreads();   // the reduction buffer below overlays the inner factor
  // D[4 q + v][i] of a 16x16 tile is element v of lane i + 16 q
  if (wx > 0) {
#pragma unroll
    for (int blk = 0; blk < LP_RB; ++blk)
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wx - 1][wr * 16 * LP_RB + 16 * blk + 4 * q + v][c * 16 + i] = macc[blk][c][v];
  }
  __syncthreads();
  if (wx == 0) {
    double* out = part + (long long)split * g.rows * R;
#pragma unroll
    for (int blk = 0; blk < LP_RB; ++blk)
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rl = wr * 16 * LP_RB + 16 * blk + 4 * q + v, col = c * 16 + i;
          float s = macc[blk][c][v];
#pragma unroll
          for (int k = 0; k < LP_WX - 1; ++k) s += red[k][rl][col];
          const int m = blockIdx.x * LP_ROWS + rl;
          if (m < g.rows && col < R) out[(long long)m * R + col] = (double)s;
        }
  }
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

// Geometry of the FP32 / BF16 kernels: 64-row blocks, outer-index ranges that are a multiple of
// LP_WX (every wave group gets the same number of outer indices), about 1024 workgroups.
MtGeom lp_geom(const int64_t dims[3], int R, int mode, int* nsplit, int* rblocks) {
  MtGeom g;
  g.I1 = (int)dims[0]; g.I2 = (int)dims[1]; g.I3 = (int)dims[2];
  g.rows = (int)dims[mode];
  g.X = (mode == 0) ? g.I2 : g.I1;
  g.Y = (mode == 2) ? g.I2 : g.I3;
  g.R = R;
  g.nct = (R + 15) / 16;
  const int rbk = (g.rows + LP_ROWS - 1) / LP_ROWS;
  const int want = (1024 + rbk - 1) / rbk;
  int xper = (g.X + want - 1) / want;
  xper = (xper + LP_WX - 1) / LP_WX * LP_WX;
  if (xper > LP_XMAX) xper = LP_XMAX;
  g.xper = xper;
  *nsplit = (g.X + xper - 1) / xper;
  *rblocks = rbk;
  return g;
}

int lp_ypad(const MtGeom& g, int kind) {
  const int kg = 4 * LP_KSUB * (kind == CPD_BF16 ? LpKind<CPD_BF16>::KPL : LpKind<CPD_F32>::KPL);
  return (g.Y + kg - 1) / kg * kg;
}

constexpr size_t LP_LDS_LIMIT = 160 * 1024 - 1024;

// Dynamic LDS of mttkrp_lp_kernel; *blds says whether the inner factor fits in it.
template <int KIND>
size_t lp_lds_bytes(const MtGeom& g, int ypad, bool* blds) {
  const size_t nc = (size_t)g.nct * 16;
  const size_t wa = ((size_t)g.xper * nc * sizeof(float) + 15) / 16 * 16;
  const size_t red = (size_t)(LP_WX - 1) * LP_ROWS * (nc + 1) * sizeof(float);
  const size_t bf = (size_t)(g.R + 1) * lp_pitch<KIND>(ypad) * sizeof(typename LpKind<KIND>::WT);
  *blds = wa + (bf > red ? bf : red) <= LP_LDS_LIMIT;
  return wa + (*blds && bf > red ? bf : red);
}

template <class TT, int KIND, int MODE, int NCT, bool VEC, bool BLDS>
cpd_status lp_go(const TT* t, const MtGeom& g, const double* Wa, const void* wbf, int ypad, double* part,
                 dim3 grid, size_t lds, hipStream_t s) {
  auto k = mttkrp_lp_kernel<TT, KIND, MODE, NCT, VEC, BLDS>;
  if (lds > 64 * 1024)
    CPD_HIP_CHECK(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, grid, dim3(LP_NT), lds, s, t, g, Wa, (const typename LpKind<KIND>::WT*)wbf, ypad, part);
  return CPD_OK;
}

template <class TT, int KIND, int MODE, int NCT>
cpd_status lp_launch(const TT* t, const MtGeom& g, const double* Wa, const void* wbf, int ypad, double* part,
                     dim3 grid, bool vec, hipStream_t s) {
  bool blds;
  const size_t lds = lp_lds_bytes<KIND>(g, ypad, &blds);
  if constexpr (MODE != 2) {
    if (vec) {
      if (blds) return lp_go<TT, KIND, MODE, NCT, true, true>(t, g, Wa, wbf, ypad, part, grid, lds, s);
      return lp_go<TT, KIND, MODE, NCT, true, false>(t, g, Wa, wbf, ypad, part, grid, lds, s);
    }
  }
  if (blds) return lp_go<TT, KIND, MODE, NCT, false, true>(t, g, Wa, wbf, ypad, part, grid, lds, s);
  return lp_go<TT, KIND, MODE, NCT, false, false>(t, g, Wa, wbf, ypad, part, grid, lds, s);
}

template <class TT, int KIND, int MODE>
cpd_status lp_launch_nct(const TT* t, const MtGeom& g, const double* Wa, const void* wbf, int ypad, double* part,
                         dim3 grid, bool vec, hipStream_t s) {
  switch (g.nct) {
    case 1: return lp_launch<TT, KIND, MODE, 1>(t, g, Wa, wbf, ypad, part, grid, vec, s);
    case 2: return lp_launch<TT, KIND, MODE, 2>(t, g, Wa, wbf, ypad, part, grid, vec, s);
    case 3: return lp_launch<TT, KIND, MODE, 3>(t, g, Wa, wbf, ypad, part, grid, vec, s);
    default: return lp_launch<TT, KIND, MODE, 4>(t, g, Wa, wbf, ypad, part, grid, vec, s);
  }
}

template <class TT, int KIND>
cpd_status lp_launch_mode(const void* T, const MtGeom& g, int mode, const double* Wa, const void* wbf, int ypad,
                          double* part, dim3 grid, bool vec, hipStream_t s) {
  const TT* t = (const TT*)T;
  if (mode == 0) return lp_launch_nct<TT, KIND, 0>(t, g, Wa, wbf, ypad, part, grid, vec, s);
  if (mode == 1) return lp_launch_nct<TT, KIND, 1>(t, g, Wa, wbf, ypad, part, grid, vec, s);
  return lp_launch_nct<TT, KIND, 2>(t, g, Wa, wbf, ypad, part, grid, vec, s);
}

}  // namespace

size_t mttkrp_ws_bytes(const int64_t dims[3], int R, int mode) {
  int ns, rb;
  const MtGeom g = mt_geom(dims, R, mode, &ns, &rb);
  Sizer z;
  z.take<double>((size_t)ns * g.rows * R);
  int ls, lr;
  const MtGeom h = lp_geom(dims, R, mode, &ls, &lr);
  const int ypad = lp_ypad(h, CPD_BF16) > lp_ypad(h, CPD_F32) ? lp_ypad(h, CPD_BF16) : lp_ypad(h, CPD_F32);
  Sizer y;
  y.take<double>((size_t)ls * h.rows * R);
  y.take<float>((size_t)h.nct * 16 * ypad);
  return z.off > y.off ? z.off : y.off;
}

cpd_status mttkrp_full(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                       int R, int mode, int compute_dtype, double* M, void* ws, size_t ws_bytes, hipStream_t s) {
  if (R < 1 || R > MT_MAXR || mode < 0 || mode > 2 || !T || !M || !W[0] || !W[1] || !W[2]) {
    set_error("mttkrp_full: bad arguments (R=%d mode=%d)", R, mode);
    return CPD_E_INVALID;
  }
  const bool lp = compute_dtype != CPD_F64;
  if (lp && !((compute_dtype == CPD_F32 && (dtype == CPD_F32 || dtype == CPD_BF16)) ||
              (compute_dtype == CPD_BF16 && dtype == CPD_BF16))) {
    set_error("mttkrp_full: compute dtype %d needs an FP32 or BF16 tensor (BF16 only for BF16), got %d",
              compute_dtype, dtype);
    return CPD_E_INVALID;
  }
  if (!ws || ws_bytes < mttkrp_ws_bytes(dims, R, mode)) {
    set_error("mttkrp_full: workspace too small");
    return CPD_E_WORKSPACE;
  }
  const double* Wa = W[mode == 0 ? 1 : 0];
  const double* Wb = W[mode == 2 ? 1 : 2];
  int ns, rb;
  const MtGeom g = lp ? lp_geom(dims, R, mode, &ns, &rb) : mt_geom(dims, R, mode, &ns, &rb);
  Arena ar(ws, ws_bytes);
  double* part = ar.take<double>((size_t)ns * g.rows * R);
  const dim3 grid(rb, ns);
  cpd_status st;
  prof_begin(CPD_PK_MTTKRP, s);
  if (!lp) {
    if (dtype == CPD_F64) launch_mt<double>(T, g, mode, Wa, Wb, part, grid, s);
    else if (dtype == CPD_F32) launch_mt<float>(T, g, mode, Wa, Wb, part, grid, s);
    else launch_mt<uint16_t>(T, g, mode, Wa, Wb, part, grid, s);
  } else {
    const int ypad = lp_ypad(g, compute_dtype), ncol = g.nct * 16;
    const long long nw = (long long)ncol * ypad;
    // vector A loads need the inner index contiguous (modes 1, 2) and every row start aligned
    const int kpl = compute_dtype == CPD_BF16 ? LpKind<CPD_BF16>::KPL : LpKind<CPD_F32>::KPL;
    const size_t esz = dtype == CPD_F32 ? 4 : 2;
    const bool vec = mode != 2 && g.Y % kpl == 0 && ((uintptr_t)T % (kpl * esz) == 0);
    if (compute_dtype == CPD_BF16) {
      uint16_t* wbf = ar.take<uint16_t>((size_t)nw);
      hipLaunchKernelGGL(mt_wb_prep_kernel<CPD_BF16>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, Wb,
                         g.Y, R, ypad, ncol, wbf);
      if ((st = lp_launch_mode<uint16_t, CPD_BF16>(T, g, mode, Wa, wbf, ypad, part, grid, vec, s))) return st;
    } else {
      float* wbf = ar.take<float>((size_t)nw);
      hipLaunchKernelGGL(mt_wb_prep_kernel<CPD_F32>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, Wb,
                         g.Y, R, ypad, ncol, wbf);
      if ((st = dtype == CPD_F32 ? lp_launch_mode<float, CPD_F32>(T, g, mode, Wa, wbf, ypad, part, grid, vec, s)
                                 : lp_launch_mode<uint16_t, CPD_F32>(T, g, mode, Wa, wbf, ypad, part, grid, vec, s)))
        return st;
    }
  }
  const long long n = (long long)g.rows * R;
  hipLaunchKernelGGL(mttkrp_reduce_kernel, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, s, part, ns, n, M);
  prof_end(CPD_PK_MTTKRP, s);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
