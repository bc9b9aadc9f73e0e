// Precision form of the payoff product: every showdown terminal of one
// player stacked into one dense contraction on the BF16 matrix cores.
//
// With hands in strength order, a showdown terminal z of player p contributes
//   out[s_p(z)][h] += b_p(h)/Z * u(z) * sign_p * sum_h' W[h][h'] r_z(h'),
//   W[h][h'] = [h, h' share no card] * sgn(s(h') - s(h))  in {-1, 0, +1},
//   r_z(h')  = b_o(h') v_o[s_o(z)][h']
// (Section 2's gradient operators, Eq. 2's payoff matrix restricted to the
// showdown leaves; W^T = -W, so player 2 uses the same W with sign -1).  All
// showdown columns r_z form Y (n x L), and C = W Y is computed as
// W Y_hi + W Y_lo with Y_hi = bf16(Y) and Y_lo = bf16(Y - Y_hi): W is exact in
// BF16, each BF16 x BF16 product is exact in FP32, the accumulation is FP32.
// The fold terminals keep their O(n) per-card evaluation (in FP64 arithmetic,
// FP32 output) in launch_gradient_fold_f32, which also zeroes the rows; the
// GEMM epilogue then adds the showdown part.  Each own sequence has at most
// one showdown terminal (checked when the tables are built), so every output
// element is updated by exactly one lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "egt_internal.h"

namespace egt {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kBM = 64;  // output hands per block
constexpr int kBN = 64;  // showdown columns per block
constexpr int kBK = 32;  // hands contracted per LDS stage
constexpr int kLdsStride = kBK + 8;  // bf16 per LDS row, padded against bank conflicts

__device__ inline unsigned short bf16_rn(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite inputs)
  return (unsigned short)(u >> 16);
}

__device__ inline float bf16_to_f32(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

struct GemmArgs {
  const unsigned short* W;  // [kpad][kpad] BF16 bits, row h, contiguous h'
  int kpad;
  int n, ld;
  int L;                    // showdown columns of the own player
  const int* col_own;       // [L] own sequence of the column
  const int* col_opp;       // [L] opponent sequence (-1 = empty sequence)
  const double* col_coef;   // [L] player-2 chips at the terminal
  const double* b_opp;      // [ld]
  const double* b_own;      // [ld]
  double scale;             // sign / Z
  const float* v_opp;       // opponent strategy [S_o][ld]
  float* out;               // own gradient [S_own][ld], fold part already written
};

__global__ __launch_bounds__(256) void show_gemm_kernel(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned short As[2][kBM * kLdsStride];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[2][kBN * kLdsStride];
  __shared__ __attribute__((aligned(16))) unsigned short Bl[2][kBN * kLdsStride];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  // staging roles: 64 rows (or columns) x 32 k = 256 threads x 8 elements
  const int srow = tid >> 2, skk = (tid & 3) * 8;
  const int j = n0 + srow;
  const bool jvalid = j < a.L;
  const float* vrow = nullptr;
  if (jvalid) {
    const int o = a.col_opp[j];
    vrow = o >= 0 ? a.v_opp + (size_t)o * a.ld : nullptr;
  }
  uint4 areg;
  float breg[8];
  auto load = [&](int ks) {
    const int k0 = ks * kBK + skk;
    areg = *(const uint4*)(a.W + (size_t)(m0 + srow) * a.kpad + k0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + e;
      float r = 0.0f;
      if (jvalid && k < a.n) r = (float)(a.b_opp[k] * (vrow ? (double)vrow[k] : 1.0));
      breg[e] = r;
    }
  };
  auto store = [&](int buf) {
    *(uint4*)&As[buf][srow * kLdsStride + skk] = areg;
    unsigned short hi[8], lo[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      hi[e] = bf16_rn(breg[e]);
      lo[e] = bf16_rn(breg[e] - bf16_to_f32(hi[e]));
    }
    uint4 ph, pl;
    ph.x = hi[0] | ((unsigned)hi[1] << 16);
    ph.y = hi[2] | ((unsigned)hi[3] << 16);
    ph.z = hi[4] | ((unsigned)hi[5] << 16);
    ph.w = hi[6] | ((unsigned)hi[7] << 16);
    pl.x = lo[0] | ((unsigned)lo[1] << 16);
    pl.y = lo[2] | ((unsigned)lo[3] << 16);
    pl.z = lo[4] | ((unsigned)lo[5] << 16);
    pl.w = lo[6] | ((unsigned)lo[7] << 16);
    *(uint4*)&Bh[buf][srow * kLdsStride + skk] = ph;
    *(uint4*)&Bl[buf][srow * kLdsStride + skk] = pl;
  };

  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  const int ksteps = a.kpad / kBK;
  load(0);
  store(0);
  __syncthreads();
  for (int ks = 0; ks < ksteps; ++ks) {
    const int buf = ks & 1;
    if (ks + 1 < ksteps) load(ks + 1);  // next stage's global loads overlap the MFMAs
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      const int koff = kk + 8 * (lane >> 5);
      const bf16x8 av = *(const bf16x8*)&As[buf][(wm + (lane & 31)) * kLdsStride + koff];
      const bf16x8 bh = *(const bf16x8*)&Bh[buf][(wn + (lane & 31)) * kLdsStride + koff];
      const bf16x8 bl = *(const bf16x8*)&Bl[buf][(wn + (lane & 31)) * kLdsStride + koff];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bl, acc, 0, 0, 0);
    }
    if (ks + 1 < ksteps) store(buf ^ 1);
    __syncthreads();
  }
  // accumulator r of lane l holds C[row][col], col = l % 32,
  // row = (r / 4) * 8 + (l / 32) * 4 + r % 4 within the wave's 32 x 32 tile
  const int jc = n0 + wn + (lane & 31);
  if (jc < a.L) {
    const double c = a.col_coef[jc] * a.scale;
    float* row = a.out + (size_t)a.col_own[jc] * a.ld;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int h = m0 + wm + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
      if (h < a.n) row[h] += (float)(c * a.b_own[h] * (double)acc[r]);
    }
  }
}

}  // namespace

// Builds W (BF16 bits) and the per-player showdown column lists on the host
// and uploads them.  Called once per game on the first precision-form use.
int ensure_mixed_tables(const egt_game* cg) {
  egt_game* g = const_cast<egt_game*>(cg);  // cached tables owned by the game
  if (g->mx.block) return EGT_OK;
  const int n = g->n;
  const int kpad = (n + kBM - 1) / kBM * kBM;
  // slot order: strength ascending; compatibility from the cards of the slots
  std::vector<unsigned short> W((size_t)kpad * kpad, 0);
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < n; ++k) {
      bool share = false;
      for (int x = 0; x < g->cph && !share; ++x)
        for (int y = 0; y < g->cph; ++y)
          if (g->slot_cards[(size_t)i * g->cph + x] == g->slot_cards[(size_t)k * g->cph + y]) share = true;
      if (share) continue;
      const int si = g->slot_strength[i], sk = g->slot_strength[k];
      W[(size_t)i * kpad + k] = sk > si ? 0x3F80 : (sk < si ? 0xBF80 : 0);
    }
  }
  std::vector<int> own[2], opp[2];
  std::vector<double> coef[2];
  for (int p = 0; p < 2; ++p) {
    const HostPlayer& hp = g->hp[p];
    for (int s = 0; s < hp.n_seq; ++s) {
      int shows = 0;
      for (int t = hp.term_begin[s]; t < hp.term_begin[s + 1]; ++t) {
        if (hp.term_kind[t] != 1) continue;
        if (++shows > 1) return fail(EGT_EINVAL, "precision form needs at most one showdown per sequence");
        own[p].push_back(s);
        opp[p].push_back(hp.term_opp[t]);
        coef[p].push_back(hp.term_coef[t]);
      }
    }
  }
  size_t bytes = sizeof(unsigned short) * W.size();
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t off_cols[2][3];
  size_t total = al(bytes);
  for (int p = 0; p < 2; ++p) {
    off_cols[p][0] = total;
    total += al(sizeof(int) * std::max<size_t>(own[p].size(), 1));
    off_cols[p][1] = total;
    total += al(sizeof(int) * std::max<size_t>(opp[p].size(), 1));
    off_cols[p][2] = total;
    total += al(sizeof(double) * std::max<size_t>(coef[p].size(), 1));
  }
  std::vector<unsigned char> staging(total, 0);
  std::memcpy(staging.data(), W.data(), bytes);
  for (int p = 0; p < 2; ++p) {
    if (!own[p].empty()) {
      std::memcpy(staging.data() + off_cols[p][0], own[p].data(), sizeof(int) * own[p].size());
      std::memcpy(staging.data() + off_cols[p][1], opp[p].data(), sizeof(int) * opp[p].size());
      std::memcpy(staging.data() + off_cols[p][2], coef[p].data(), sizeof(double) * coef[p].size());
    }
  }
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, total);
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc (precision tables): ") + hipGetErrorString(e));
  e = hipMemcpy(dev, staging.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e, "upload of precision tables");
  }
  g->mx.kpad = kpad;
  g->mx.W = (const unsigned short*)dev;
  for (int p = 0; p < 2; ++p) {
    g->mx.L[p] = (int)own[p].size();
    g->mx.col_own[p] = (const int*)((unsigned char*)dev + off_cols[p][0]);
    g->mx.col_opp[p] = (const int*)((unsigned char*)dev + off_cols[p][1]);
    g->mx.col_coef[p] = (const double*)((unsigned char*)dev + off_cols[p][2]);
  }
  g->mx.block = dev;
  return EGT_OK;
}

hipError_t launch_show_gemm(const egt_game* g, int player, const float* v_opp, float* grad_out, hipStream_t s) {
  const MixedTables& m = g->mx;
  if (m.L[player] == 0) return hipSuccess;
  GemmArgs a;
  a.W = m.W;
  a.kpad = m.kpad;
  a.n = g->n;
  a.ld = g->ld;
  a.L = m.L[player];
  a.col_own = m.col_own[player];
  a.col_opp = m.col_opp[player];
  a.col_coef = m.col_coef[player];
  a.b_opp = g->dp[1 - player].belief;
  a.b_own = g->dp[player].belief;
  a.scale = (player == 0 ? 1.0 : -1.0) / g->Z;
  a.v_opp = v_opp;
  a.out = grad_out;
  const dim3 grid((unsigned)((a.L + kBN - 1) / kBN), (unsigned)(m.kpad / kBM));
  hipLaunchKernelGGL(show_gemm_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gradient_mixed(const egt_game* g, int player, const float* v_opp, float* grad_out, hipStream_t s) {
  hipError_t e = launch_gradient_fold_f32(g, player, v_opp, grad_out, s);
  if (e != hipSuccess) return e;
  return launch_show_gemm(g, player, v_opp, grad_out, s);
}

}  // namespace egt
