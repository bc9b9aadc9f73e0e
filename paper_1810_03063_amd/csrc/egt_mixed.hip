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
// The fold terminals keep their O(n) per-card evaluation (in FP32) in
// launch_gradient_fold_f32, which also zeroes the other rows; the
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

constexpr int kTile = 32;     // output hands x showdown columns per block (one 32x32 MFMA tile)
constexpr int kKWaves = 16;   // waves per block, each contracting every 16th k-step of 16 hands
constexpr int kBatch = 3;     // k-steps whose operands a wave loads before multiplying
constexpr int kRedStride = kTile + 1;
constexpr int kTiledMinColumns = 512;  // from this many showdown columns on, the tiled GEMM

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Two floats to BF16, round to nearest with ties to even (gfx950 converts a
// pair in one instruction), packed low element first.
__device__ inline unsigned bf16x2_rn(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2v));
}

// Eight FP32 reaches split into BF16 hi = bf16(r) and lo = bf16(r - hi).
__device__ inline void split8(const float r[8], bf16x8& hi, bf16x8& lo) {
  unsigned h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = bf16x2_rn(r[2 * e], r[2 * e + 1]);
    l[e] = bf16x2_rn(r[2 * e] - __uint_as_float(h[e] << 16), r[2 * e + 1] - __uint_as_float(h[e] & 0xffff0000u));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

struct GemmArgs {
  const unsigned short* W;  // [ld][ld] BF16 bits, row h, contiguous h'
  int n, ld;
  int L;                    // showdown columns of the own player
  const int* col_own;       // [L] own sequence of the column
  const int* col_opp;       // [L] opponent sequence (-1 = empty sequence)
  const double* col_coef;   // [L] player-2 chips at the terminal
  const float* b_opp32;     // [ld] opponent prior in FP32
  const double* b_own;      // [ld]
  double scale;             // sign / Z
  const float* v_opp;       // opponent strategy [S_o][ld]
  float* out;               // own gradient [S_own][ld], fold part already written
};

// One 32 x 32 output tile (hands m0.., columns n0..) per block.  The k-steps
// of 16 hands are dealt round-robin to the 16 waves; each wave loads the
// operands of kBatch steps straight into registers (no reuse inside a block,
// so no LDS staging), forms the FP32 reach, splits it into BF16 hi + lo and
// issues two 32x32x16 MFMAs per step.  The 16 partial tiles are summed
// through LDS in wave order, and one lane per output element applies the
// epilogue.
// Operand layouts of v_mfma_f32_32x32x16_bf16 (lane l, element e < 8):
//   A[l % 32][8 (l / 32) + e], B[8 (l / 32) + e][l % 32];
//   accumulator r: row (r / 4) 8 + (l / 32) 4 + r % 4, column l % 32.
__global__ __launch_bounds__(64 * kKWaves) void show_gemm_kernel(GemmArgs a) {
  __shared__ float red[kKWaves * kTile * kRedStride];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int half = lane >> 5, l32 = lane & 31;
  const int col = n0 + l32;
  const float* vrow = nullptr;
  const bool cvalid = col < a.L;
  if (cvalid) {
    const int o = a.col_opp[col];
    vrow = o >= 0 ? a.v_opp + (size_t)o * a.ld : nullptr;
  }
  const unsigned short* wrow = a.W + (size_t)(m0 + l32) * a.ld + 8 * half;
  const int nk = a.ld / 16;

  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int base = wave; base < nk; base += kKWaves * kBatch) {
    uint4 av[kBatch];
    float4 v0[kBatch], v1[kBatch], b0[kBatch], b1[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int ks = base + u * kKWaves;
      av[u] = make_uint4(0u, 0u, 0u, 0u);
      v0[u] = v1[u] = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
      b0[u] = b1[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (ks < nk) {
        const int k0 = ks * 16 + 8 * half;
        av[u] = *(const uint4*)(wrow + ks * 16);
        if (cvalid) {
          if (vrow) {
            v0[u] = *(const float4*)(vrow + k0);
            v1[u] = *(const float4*)(vrow + k0 + 4);
          }
          b0[u] = *(const float4*)(a.b_opp32 + k0);
          b1[u] = *(const float4*)(a.b_opp32 + k0 + 4);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (base + u * kKWaves >= nk) break;  // uniform within the wave
      // FP32 reach of the 8 hands, split into BF16 hi + lo
      const float r[8] = {b0[u].x * v0[u].x, b0[u].y * v0[u].y, b0[u].z * v0[u].z, b0[u].w * v0[u].w,
                          b1[u].x * v1[u].x, b1[u].y * v1[u].y, b1[u].z * v1[u].z, b1[u].w * v1[u].w};
      bf16x8 hi, lo;
      split8(r, hi, lo);
      const bf16x8 am = *(const bf16x8*)&av[u];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, hi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, lo, acc, 0, 0, 0);
    }
  }
  // partial tiles to LDS as red[wave][column][row]
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = (r >> 2) * 8 + half * 4 + (r & 3);
    red[(wave * kTile + l32) * kRedStride + row] = acc[r];
  }
  __syncthreads();
  // one lane per output element: hands fastest, so each row is written coalesced
  const int h = m0 + (tid & 31), cl = tid >> 5, j = n0 + cl;
  if (j < a.L && h < a.n) {
    float sum = 0.0f;
#pragma unroll
    for (int w = 0; w < kKWaves; ++w) sum += red[(w * kTile + cl) * kRedStride + (tid & 31)];
    const double c = a.col_coef[j] * a.scale;
    float* row = a.out + (size_t)a.col_own[j] * a.ld;
    row[h] += (float)(c * a.b_own[h] * (double)sum);
  }
}

// Many showdown columns (large trees): a tiled GEMM with operand reuse.
// Block = 128 output hands x 64 columns, four waves, wave w owning rows
// 32 w .. 32 w + 31 of the tile as two 32 x 32 MFMA tiles.  K (the opponent's
// hands) advances in steps of kTK = 32 (ld is a multiple of 32): the block
// stages W[128 x 32] and the column reaches split into BF16 hi and lo
// ([64 columns x 32], k contiguous) in two LDS buffers, and the global loads
// run two steps ahead in registers, so each load has two steps of work to
// land behind.  The opponent's FP32 prior is staged in LDS once.  The hi and
// lo products accumulate in separate tiles (independent MFMA chains), added
// in the epilogue, which goes through LDS so that every output row is updated
// with coalesced accesses.  Tiles are numbered column block major and dealt to
// the XCDs in contiguous ranges, so the row blocks that share a column block's
// reaches meet in one L2.
constexpr int kTM = 128, kTN = 64, kTK = 32;
constexpr int kTKS = kTK + 8;  // LDS row stride (BF16 elements) of the staged operands
constexpr int kTCS = kTM + 1;  // LDS column stride (floats) of the output tile

struct TiledStage {
  unsigned short a[kTM * kTKS];   // W rows, k contiguous
  unsigned short bh[kTN * kTKS];  // reach hi, per column, k contiguous
  unsigned short bl[kTN * kTKS];  // reach lo
};
static_assert(sizeof(TiledStage) % 16 == 0, "the stages and the prior stay 16-byte aligned");
static_assert(kTCS * kTN * sizeof(float) <= 2 * sizeof(TiledStage), "the output tile fits the stages");

size_t tiled_lds_bytes(int ld) { return 2 * sizeof(TiledStage) + sizeof(float) * (size_t)ld; }

// Launch index -> tile, each XCD (launch indices go round-robin over the 8
// XCDs) taking a contiguous range of tiles.
__device__ inline int tile_of_launch(int b, int total) {
  const int q = total / 8, r = total % 8;
  const int x = b % 8, j = b / 8;
  return x * q + min(x, r) + j;
}

__global__ __launch_bounds__(256) void show_gemm_tiled_kernel(GemmArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  TiledStage* st = (TiledStage*)smem;                     // [2]
  float* bopp = (float*)(smem + 2 * sizeof(TiledStage));  // [ld]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const int n_rb = (a.ld + kTM - 1) / kTM;
  const int t = tile_of_launch((int)blockIdx.x, (int)gridDim.x);
  const int m0 = (t % n_rb) * kTM, n0 = (t / n_rb) * kTN;
  const int nst = a.ld / kTK;

  // per thread and step: 16 k of one W row, 8 k of one column's reach
  const int arow = tid >> 1, ak = (tid & 1) * 16;
  const bool arow_ok = m0 + arow < a.ld;
  const unsigned short* wsrc = a.W + (size_t)(m0 + arow) * a.ld + ak;
  const int bcol = tid >> 2, bk = (tid & 3) * 8;
  const int jcol = n0 + bcol;
  const bool bcol_ok = jcol < a.L;
  const float* vsrc = nullptr;
  if (bcol_ok) {
    const int o = a.col_opp[jcol];
    vsrc = o >= 0 ? a.v_opp + (size_t)o * a.ld : nullptr;
  }
  for (int i = tid; i < a.ld; i += 256) bopp[i] = a.b_opp32[i];
  struct StepRegs {
    uint4 a0, a1;
    float4 v0, v1;
  };
  auto load_step = [&](StepRegs& q, int s) {
    const int k0 = s * kTK;
    q.a0 = q.a1 = make_uint4(0u, 0u, 0u, 0u);
    if (arow_ok) {
      q.a0 = *(const uint4*)(wsrc + k0);
      q.a1 = *(const uint4*)(wsrc + k0 + 8);
    }
    // a column past the last one has reach 0; the empty sequence has v = 1
    const float vfill = bcol_ok ? 1.0f : 0.0f;
    q.v0 = q.v1 = make_float4(vfill, vfill, vfill, vfill);
    if (vsrc) {
      q.v0 = *(const float4*)(vsrc + k0 + bk);
      q.v1 = *(const float4*)(vsrc + k0 + bk + 4);
    }
  };
  auto store_step = [&](const StepRegs& q, int s, TiledStage& d) {
    *(uint4*)&d.a[arow * kTKS + ak] = q.a0;
    *(uint4*)&d.a[arow * kTKS + ak + 8] = q.a1;
    const int kb = s * kTK + bk;
    const float4 b0 = *(const float4*)&bopp[kb], b1 = *(const float4*)&bopp[kb + 4];
    const float r[8] = {b0.x * q.v0.x, b0.y * q.v0.y, b0.z * q.v0.z, b0.w * q.v0.w,
                        b1.x * q.v1.x, b1.y * q.v1.y, b1.z * q.v1.z, b1.w * q.v1.w};
    bf16x8 hi, lo;
    split8(r, hi, lo);
    *(bf16x8*)&d.bh[bcol * kTKS + bk] = hi;
    *(bf16x8*)&d.bl[bcol * kTKS + bk] = lo;
  };

  f32x16 acc_hi[2], acc_lo[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc_hi[c][r] = 0.0f;
      acc_lo[c][r] = 0.0f;
    }
  const int arow_w = (wave * 32 + l32) * kTKS + 8 * half;  // this lane's A operand row
  const int bcol_w = l32 * kTKS + 8 * half;                // this lane's B operand column (tile 0)
  auto multiply = [&](const TiledStage& c) {
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 16) {
      const bf16x8 am = *(const bf16x8*)&c.a[arow_w + kk];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const bf16x8 bh = *(const bf16x8*)&c.bh[bcol_w + 32 * ct * kTKS + kk];
        const bf16x8 bl = *(const bf16x8*)&c.bl[bcol_w + 32 * ct * kTKS + kk];
        acc_hi[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc_hi[ct], 0, 0, 0);
        acc_lo[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bl, acc_lo[ct], 0, 0, 0);
      }
    }
  };
  // Step s is multiplied from st[s & 1] while step s + 1 waits in registers
  // for the other buffer and step s + 2 is being loaded.
  StepRegs q0, q1;
  load_step(q0, 0);
  __syncthreads();  // the prior is staged
  store_step(q0, 0, st[0]);
  if (nst > 1) load_step(q0, 1);
  __syncthreads();
  int s = 0;
  for (; s + 1 < nst; s += 2) {
    // st[0] holds step s, q0 step s + 1
    if (s + 2 < nst) load_step(q1, s + 2);
    multiply(st[0]);
    store_step(q0, s + 1, st[1]);
    __syncthreads();
    // st[1] holds step s + 1, q1 step s + 2
    if (s + 3 < nst) load_step(q0, s + 3);
    multiply(st[1]);
    if (s + 2 < nst) store_step(q1, s + 2, st[0]);
    __syncthreads();
  }
  if (s < nst) {  // an odd number of steps ends in st[0]
    multiply(st[0]);
    __syncthreads();  // the output tile below overwrites the stages
  }
  // output tile through LDS as ct[column][row] (the stage is free now)
  float* ct = (float*)smem;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wave * 32 + (r >> 2) * 8 + half * 4 + (r & 3);
      const int col = 32 * c + l32;
      ct[col * kTCS + row] = acc_hi[c][r] + acc_lo[c][r];
    }
  __syncthreads();
  // Each thread updates one hand in kEpi columns per pass, with every load of
  // a pass issued before its first store (a store could alias a later load,
  // so the compiler would otherwise serialise the read-modify-writes).
  constexpr int kEpi = 16;
  constexpr int kColsPerSweep = 256 / kTM;  // columns covered by one sweep of the threads
  const int row = tid % kTM, h = m0 + row;
  const bool hok = h < a.n;
  const double bo = hok ? a.b_own[h] : 0.0;
#pragma unroll 1
  for (int pass = 0; pass < kTN / (kColsPerSweep * kEpi); ++pass) {
    int own[kEpi];
    double cf[kEpi];
#pragma unroll
    for (int u = 0; u < kEpi; ++u) {
      const int j = n0 + tid / kTM + kColsPerSweep * (pass * kEpi + u);
      own[u] = -1;
      cf[u] = 0.0;
      if (hok && j < a.L) {
        own[u] = a.col_own[j];
        cf[u] = a.col_coef[j];
      }
    }
    float cur[kEpi];
#pragma unroll
    for (int u = 0; u < kEpi; ++u) cur[u] = own[u] >= 0 ? a.out[(size_t)own[u] * a.ld + h] : 0.0f;
#pragma unroll
    for (int u = 0; u < kEpi; ++u) {
      if (own[u] < 0) continue;
      const int col = tid / kTM + kColsPerSweep * (pass * kEpi + u);
      const double c = cf[u] * a.scale;
      a.out[(size_t)own[u] * a.ld + h] = cur[u] + (float)(c * bo * (double)ct[col * kTCS + row]);
    }
  }
}

}  // namespace

// W (BF16 bits) and the per-player showdown column lists as one host image:
// W at 0, then per player the FP32 prior (off[p][3]) and the column lists
// (own sequence off[p][0], opponent sequence off[p][1], chips off[p][2]).
int mixed_tables_image(const egt_game* g, std::vector<unsigned char>& img, size_t off[2][4]) {
  if (g->general) return fail(EGT_EINVAL, "the precision form needs a river endgame");
  const int n = g->n;
  const int kpad = g->ld;  // rows and columns padded like every vector
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
  // FP32 copies of the priors (the reach b v is formed in FP32)
  std::vector<float> b32[2];
  for (int p = 0; p < 2; ++p) b32[p].assign(g->hbelief[p].begin(), g->hbelief[p].end());
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t wbytes = sizeof(unsigned short) * W.size();
  size_t total = al(wbytes);
  for (int p = 0; p < 2; ++p) {
    off[p][3] = total;
    total += al(sizeof(float) * b32[p].size());
  }
  for (int p = 0; p < 2; ++p) {
    off[p][0] = total;
    total += al(sizeof(int) * std::max<size_t>(own[p].size(), 1));
    off[p][1] = total;
    total += al(sizeof(int) * std::max<size_t>(opp[p].size(), 1));
    off[p][2] = total;
    total += al(sizeof(double) * std::max<size_t>(coef[p].size(), 1));
  }
  img.assign(total, 0);
  std::memcpy(img.data(), W.data(), wbytes);
  for (int p = 0; p < 2; ++p) {
    std::memcpy(img.data() + off[p][3], b32[p].data(), sizeof(float) * b32[p].size());
    if (!own[p].empty()) {
      std::memcpy(img.data() + off[p][0], own[p].data(), sizeof(int) * own[p].size());
      std::memcpy(img.data() + off[p][1], opp[p].data(), sizeof(int) * opp[p].size());
      std::memcpy(img.data() + off[p][2], coef[p].data(), sizeof(double) * coef[p].size());
    }
  }
  for (int p = 0; p < 2; ++p) const_cast<egt_game*>(g)->hp[p].n_show_cols = (int)own[p].size();
  return EGT_OK;
}

int mixed_tables_upload(egt_game* g, const std::vector<unsigned char>& img, const size_t off[2][4], void* dev,
                        bool owned, hipStream_t s) {
  EGT_HIP(hipMemcpyAsync(dev, img.data(), img.size(), hipMemcpyHostToDevice, s));
  g->mx.kpad = g->ld;
  g->mx.W = (const unsigned short*)dev;
  for (int p = 0; p < 2; ++p) {
    g->mx.L[p] = g->hp[p].n_show_cols;
    g->mx.col_own[p] = (const int*)((unsigned char*)dev + off[p][0]);
    g->mx.col_opp[p] = (const int*)((unsigned char*)dev + off[p][1]);
    g->mx.col_coef[p] = (const double*)((unsigned char*)dev + off[p][2]);
    g->mx.belief32[p] = (const float*)((unsigned char*)dev + off[p][3]);
  }
  g->mx.owned = owned;
  g->mx.block = dev;
  return EGT_OK;
}

// Builds and uploads the precision-form tables once per game, on first use
// (synchronous upload).
int ensure_mixed_tables(const egt_game* cg) {
  egt_game* g = const_cast<egt_game*>(cg);  // cached tables owned by the game
  if (g->mx.block) return EGT_OK;
  std::vector<unsigned char> img;
  size_t off[2][4];
  int rc = mixed_tables_image(g, img, off);
  if (rc) return rc;
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, img.size());
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc (precision tables): ") + hipGetErrorString(e));
  e = hipMemcpy(dev, img.data(), img.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e, "upload of precision tables");
  }
  // the image is on the device now: point the tables at it (no second copy)
  g->mx.kpad = g->ld;
  g->mx.W = (const unsigned short*)dev;
  for (int p = 0; p < 2; ++p) {
    g->mx.L[p] = g->hp[p].n_show_cols;
    g->mx.col_own[p] = (const int*)((unsigned char*)dev + off[p][0]);
    g->mx.col_opp[p] = (const int*)((unsigned char*)dev + off[p][1]);
    g->mx.col_coef[p] = (const double*)((unsigned char*)dev + off[p][2]);
    g->mx.belief32[p] = (const float*)((unsigned char*)dev + off[p][3]);
  }
  g->mx.owned = true;
  g->mx.block = dev;
  return EGT_OK;
}

hipError_t launch_show_gemm(const egt_game* g, int player, const float* v_opp, float* grad_out, hipStream_t s) {
  const MixedTables& m = g->mx;
  if (m.L[player] == 0) return hipSuccess;
  GemmArgs a;
  a.W = m.W;
  a.n = g->n;
  a.ld = g->ld;
  a.L = m.L[player];
  a.col_own = m.col_own[player];
  a.col_opp = m.col_opp[player];
  a.col_coef = m.col_coef[player];
  a.b_opp32 = m.belief32[1 - player];
  a.b_own = g->dp[player].belief;
  a.scale = (player == 0 ? 1.0 : -1.0) / g->Z;
  a.v_opp = v_opp;
  a.out = grad_out;
  if (a.L >= kTiledMinColumns) {
    // enough columns for operand reuse to pay: the tiled form
    const unsigned tiles = (unsigned)(((a.L + kTN - 1) / kTN) * ((g->ld + kTM - 1) / kTM));
    hipLaunchKernelGGL(show_gemm_tiled_kernel, dim3(tiles), dim3(256), tiled_lds_bytes(g->ld), s, a);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((a.L + kTile - 1) / kTile), (unsigned)(g->ld / kTile));
  hipLaunchKernelGGL(show_gemm_kernel, grid, dim3(64 * kKWaves), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gradient_mixed(const egt_game* g, int player, const float* v_opp, float* grad_out, hipStream_t s) {
  hipError_t e = launch_gradient_fold_f32(g, player, v_opp, grad_out, s);
  if (e != hipSuccess) return e;
  return launch_show_gemm(g, player, v_opp, grad_out, s);
}

}  // namespace egt
