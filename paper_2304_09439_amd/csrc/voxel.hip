// Voxel-embedding LOCC variant (Sec. III, appendix "Architecture Details").
//
// Shape encoder (once per shape, at upload; float32 arithmetic, float64 grid
// assignment): cell_sort_kernel orders each shape's points by grid cell;
// point_mlp_kernel runs the per-point MLP over chunks of 64 points in that
// order (layers 2-3 on the matrix cores) and keeps the channel-wise max per
// grid cell (an atomic max per run of equal cells, on the bit patterns, which
// order like the values for the non-negative ReLU outputs);
// conv_kernel runs every convolution and transposed convolution of the
// U-Net as an implicit GEMM on the matrix cores (the skip concatenation read
// from two inputs); global_kernel takes max and mean over the bottleneck cells;
// embed_kernel maps [last layer, global feature] to the 16-float embedding;
// consts_kernel writes the float64 cell size and margin of each shape.
//
// Predictor, two launches.  select_kernel: one wave per pair validates it,
// puts it in canonical order, computes the float64 relative pose
// (wave-uniform), runs each object's 216 cell tests (centres formed in
// registers; float64, fixed order, contraction off) as four 64-lane ballots
// and the means of the selected cells' embeddings (lane = 4 features x cell
// residue mod 16, the float4 loads of both objects issued together, summed
// across the residues by shuffles), and writes both objects' predictor input
// rows to the workspace; with small register use many waves are in flight
// to hide the load latency.  mlp_kernel: 32 pairs per workgroup of eight waves run the
// per-object MLP on the 64 rows, the pair max, the pair MLP and the output
// layer in float32, activations in one LDS buffer that each layer
// overwrites after all its reads; every thread owns one output column of a
// layer for a quarter of the rows, reading the weights [in][out] from L2
// (coalesced) and the rows from LDS as broadcasts.
#include "geometry.h"
#include "voxel.h"

namespace locc {
namespace vox {
namespace {

__device__ __forceinline__ float relu(float x) { return x > 0.f ? x : 0.f; }

// Grid cell of a stored point (float64, the order of the reading).
__device__ __forceinline__ int cell_of(float x, float y, float z, const Shape& sh) {
#pragma clang fp contract(off)
  const float p[3] = {x, y, z};
  int idx = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double lo = sh.lo[k], hi = sh.hi[k];
    const double ext = hi - lo;
    int i = 0;
    if (ext > 0.0) {
      const double t = (((double)p[k] - lo) * (double)kM) / ext;
      i = (int)__builtin_floor(t);
      i = i < 0 ? 0 : (i > kM - 1 ? kM - 1 : i);
    }
    idx = idx * kM + i;
  }
  return idx;
}

// Counting sort of each shape's points by grid cell (a workgroup per shape):
// the cell histogram, its exclusive scan, then each point's slot from its
// cell's cursor.  The order within a cell depends on the timing of the LDS
// atomics; the cell max built from it does not.
__global__ __launch_bounds__(1024) void cell_sort_kernel(const Shape* shapes, const float* xyz, int64_t n_points,
                                                          int32_t* order, uint8_t* cells) {
  __shared__ int hist[kCells];
  const Shape sh = shapes[blockIdx.x];
  const int t = threadIdx.x;
  auto cell_at = [&](int i) {
    const int64_t r = (int64_t)sh.off + i;
    return cell_of(xyz[r], xyz[n_points + r], xyz[2 * n_points + r], sh);
  };
  for (int c = t; c < kCells; c += 1024) hist[c] = 0;
  __syncthreads();
  for (int i = t; i < sh.n; i += 1024) atomicAdd(&hist[cell_at(i)], 1);
  __syncthreads();
  if (t == 0) {  // exclusive scan: hist[c] becomes the first slot of cell c
    int run = 0;
    for (int c = 0; c < kCells; ++c) {
      const int h = hist[c];
      hist[c] = run;
      run += h;
    }
  }
  __syncthreads();
  for (int i = t; i < sh.n; i += 1024) {
    const int c = cell_at(i);
    const int slot = atomicAdd(&hist[c], 1);
    order[sh.off + slot] = i;
    cells[sh.off + slot] = (uint8_t)c;
  }
}

constexpr int kPts = 64;  // points per workgroup of the point MLP

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Per-point MLP 3 -> 256 -> 256 -> 256 over 64 points, taken in cell order,
// and the cell max.
// Layer 1 on the vector units (a wave per 64 channels, a lane per point);
// layers 2 and 3 on the matrix cores (v_mfma_f32_32x32x2f32, bias as the
// accumulator's start): wave w owns output channels [64 w, 64 w + 64), two
// 32-channel tiles over the two 32-point tiles, its A operands the rows of
// the transposed weights Wt[in][out] (coalesced, four steps ahead), its B
// operands the activations, kept channel-major in LDS (HT[c][p]: a step
// reads two rows of 32 points).  The last layer's outputs go to LDS too;
// a thread per channel then walks the 64 points, whose cells come in runs,
// and issues one atomic max per run.  Lane layouts as in conv_kernel below.
__global__ __launch_bounds__(256) void point_mlp_kernel(PackedNet w, const Shape* shapes, const float* xyz,
                                                         int64_t n_points, const int32_t* order,
                                                         const uint8_t* cells, float* grid) {
  __shared__ float X[kPts][4];
  __shared__ int cell[kPts];
  __shared__ float HT[kH][kPts + 1];  // padded: the pooling walk reads a column
  const int s = blockIdx.y;
  const Shape sh = shapes[s];
  const int base = blockIdx.x * kPts;
  if (base >= sh.n) return;  // uniform
  const int np = sh.n - base < kPts ? sh.n - base : kPts;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5, l32 = lane & 31;
  if (t < kPts) {
    float x = 0.f, y = 0.f, z = 0.f;
    int c = -1;
    if (t < np) {
      const int64_t q = (int64_t)sh.off + base + t;
      const int64_t r = (int64_t)sh.off + order[q];
      x = xyz[r];
      y = xyz[n_points + r];
      z = xyz[2 * n_points + r];
      c = cells[q];
    }
    X[t][0] = x;
    X[t][1] = y;
    X[t][2] = z;
    cell[t] = c;
  }
  __syncthreads();
  {  // layer 1: lane = point, the wave's 64 channels in turn
    const float x = X[lane][0], y = X[lane][1], z = X[lane][2];
    for (int k = 0; k < 64; ++k) {
      const int o = wave * 64 + k;
      HT[o][lane] = relu(((w.P1[3 * o] * x + w.P1[3 * o + 1] * y) + w.P1[3 * o + 2] * z) + w.p1[o]);
    }
  }
  __syncthreads();
  f32x16 acc[2][2];  // [channel tile][point tile]
  for (int layer = 0; layer < 2; ++layer) {
    const float* Wt = (layer ? w.P3t : w.P2t) + (size_t)g * kH + wave * 64 + l32;
    const float* bias = (layer ? w.p3 : w.p2) + wave * 64 + 4 * g;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float b = bias[32 * ot + 8 * (r >> 2) + (r & 3)];
        acc[ot][0][r] = b;
        acc[ot][1][r] = b;
      }
    constexpr int kAhead = 4;
    float ar[kAhead][2];
#pragma unroll
    for (int d = 0; d < kAhead; ++d)
#pragma unroll
      for (int ot = 0; ot < 2; ++ot) ar[d][ot] = Wt[(size_t)2 * d * kH + 32 * ot];
    for (int k = 0; k < kH; k += 2 * kAhead) {
#pragma unroll
      for (int d = 0; d < kAhead; ++d) {
        const int kk = k + 2 * d;
        const float b0 = HT[kk + g][l32], b1 = HT[kk + g][32 + l32];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
          acc[ot][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[d][ot], b0, acc[ot][0], 0, 0, 0);
          acc[ot][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[d][ot], b1, acc[ot][1], 0, 0, 0);
        }
        const int kn = kk + 2 * kAhead;
        if (kn < kH) {
#pragma unroll
          for (int ot = 0; ot < 2; ++ot) ar[d][ot] = Wt[(size_t)kn * kH + 32 * ot];
        }
      }
    }
    __syncthreads();  // every wave has read HT
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
      for (int pt = 0; pt < 2; ++pt)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          HT[wave * 64 + 32 * ot + 8 * (r >> 2) + 4 * g + (r & 3)][32 * pt + l32] = relu(acc[ot][pt][r]);
    __syncthreads();
  }
  // max over each run of equal cells (the grid starts at 0 and the outputs are >= 0)
  unsigned int* gp = reinterpret_cast<unsigned int*>(grid) + ((size_t)s * kH + t) * kCells;
  int cur = cell[0];
  float m = 0.f;
  for (int p = 0; p < np; ++p) {
    const int c = cell[p];  // uniform
    if (c != cur) {
      atomicMax(gp + cur, __float_as_uint(m));
      cur = c;
      m = 0.f;
    }
    m = fmaxf(m, HT[t][p]);
  }
  atomicMax(gp + cur, __float_as_uint(m));
}

// Convolutions and transposed convolutions of the U-Net as implicit GEMMs on
// the matrix cores (v_mfma_f32_32x32x2f32): out[s][o][x] = ReLU(b[o] +
// sum_{u, c} W[o][c][u] in(c, u, s, x)) over the 27 taps u and the input
// channels c (the skip concatenation read from two inputs), in(c, u, s, x) =
// input c of shape s at x + u - pad (conv) or x - u + pad (transposed), 0
// outside the grid.  A workgroup owns 32 output channels x 32 output
// positions; its eight waves take an eighth of the channels each, NP pairs
// of them, over all 27 taps, tap-major: a tap's grid offset and bounds test
// are formed once per lane and serve its NP steps, and the next tap's
// operands load while the current tap's NP products issue.  The weights come
// transposed, Wt[u][c][o], so that a step's A operand is two coalesced rows.
// The waves' 32 x 32 partial sums meet in LDS and are added in wave order (a
// fixed order: a launch is reproducible bit for bit).  Lane layouts of
// 32x32x2: A[i][k] and B[k][j] with i, j = l % 32 and k = l / 32 (here the
// channel parity); D[i][j] with j = l % 32 and i = 8 (r / 4) + 4 (l / 32) +
// r % 4 for register r.
struct ConvArgs {
  const float* in1;  // [S][c1][D^3]
  int c1;
  const float* in2;  // [S][c2][D^3] (the concatenated skip), or null with c2 = 0
  int c2;
  const float* Wt;   // [27][c1 + c2][O]
  const float* b;    // [O]
  float* out;        // [S][O][Do^3]
  int O, D, Do, pad, transposed, n_shapes;
};

constexpr int kConvWaves = 8;

template <int NP>  // channel pairs per wave: (c1 + c2) = 16 NP
__global__ __launch_bounds__(64 * kConvWaves) void conv_kernel(ConvArgs A) {
  __shared__ float part[kConvWaves][32][33];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 5, l32 = lane & 31;
  const int D = A.D, Do = A.Do, D3 = D * D * D, Do3 = Do * Do * Do;
  const int N = A.n_shapes * Do3, C = A.c1 + A.c2, O = A.O;
  const int n0 = blockIdx.x * 32, o0 = blockIdx.y * 32;
  // this lane's output position (B column)
  const int n = n0 + l32;
  const bool live = n < N;
  const int sh = live ? n / Do3 : 0, x = live ? n % Do3 : 0;
  const int x0 = x / (Do * Do), x1 = (x / Do) % Do, x2 = x % Do;
  // this wave's channels c_begin + 2 j + g, all from one input (c1 is a multiple of 2 NP)
  const int c_begin = wave * 2 * NP;
  const float* src = c_begin < A.c1 ? A.in1 + ((size_t)sh * A.c1 + c_begin + g) * D3
                                    : A.in2 + ((size_t)sh * A.c2 + (c_begin - A.c1) + g) * D3;
  const float* wt = A.Wt + (size_t)(c_begin + g) * O + o0 + l32;
  const size_t tap_stride = (size_t)C * O;
  // The loads are unconditional (a tap outside the grid reads the channel's
  // first value) and the bound test selects 0 at the product, so that no
  // branch splits the loads of a tap and the waits stay per operand.
  auto load = [&](int u, float (&a)[NP], float (&b)[NP]) -> bool {
    const int u0 = u / 9, u1 = (u / 3) % 3, u2 = u % 3;
    const int y0 = A.transposed ? x0 - u0 + A.pad : x0 + u0 - A.pad;
    const int y1 = A.transposed ? x1 - u1 + A.pad : x1 + u1 - A.pad;
    const int y2 = A.transposed ? x2 - u2 + A.pad : x2 + u2 - A.pad;
    const bool ok = live && y0 >= 0 && y0 < D && y1 >= 0 && y1 < D && y2 >= 0 && y2 < D;
    const float* sp = src + (ok ? (y0 * D + y1) * D + y2 : 0);
    const float* wp = wt + (size_t)u * tap_stride;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      a[j] = wp[(size_t)2 * j * O];
      b[j] = sp[2 * j * D3];
    }
    return ok;
  };
  f32x16 acc = f32x16{};
  float a0[NP], b0[NP], a1[NP], b1[NP];
  // taps in pairs (u, u + 1) for u = 0, 2, ..., 24, then tap 26; no branch
  // around a load, so each product waits only for its own operands
  bool ok0 = load(0, a0, b0);
  for (int u = 0; u < 26; u += 2) {
    const bool ok1 = load(u + 1, a1, b1);
#pragma unroll
    for (int j = 0; j < NP; ++j)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[j], ok0 ? b0[j] : 0.f, acc, 0, 0, 0);
    ok0 = load(u + 2, a0, b0);
#pragma unroll
    for (int j = 0; j < NP; ++j)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[j], ok1 ? b1[j] : 0.f, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < NP; ++j)
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[j], ok0 ? b0[j] : 0.f, acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 16; ++r) part[wave][8 * (r >> 2) + 4 * g + (r & 3)][l32] = acc[r];
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += 64 * kConvWaves) {
    const int i = e >> 5, j = e & 31;   // output channel o0 + i, position n0 + j
    const int nn = n0 + j;
    if (nn >= N) continue;
    float v = A.b[o0 + i];
#pragma unroll
    for (int w = 0; w < kConvWaves; ++w) v += part[w][i][j];
    const int s2 = nn / Do3, xx = nn % Do3;
    A.out[((size_t)s2 * O + o0 + i) * Do3 + xx] = relu(v);
  }
}

__global__ __launch_bounds__(kC) void global_kernel(const float* c4, float* glob) {
  const int s = blockIdx.x, c = threadIdx.x;
  const float* src = c4 + ((size_t)s * kC + c) * kB;
  float m = src[0], sum = 0.f;
  for (int x = 0; x < kB; ++x) {
    m = src[x] > m ? src[x] : m;
    sum += src[x];
  }
  glob[(size_t)s * 2 * kC + c] = m;
  glob[(size_t)s * 2 * kC + kC + c] = sum / (float)kB;
}

// E[s][cell][f] = l[f] + L[f] . [d4[s][:][cell], glob[s]]
__global__ __launch_bounds__(256) void embed_kernel(PackedNet w, const float* d4, const float* glob, float* emb,
                                                    int n_shapes) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= n_shapes * kCells * kF) return;
  const int f = id % kF, cell = (id / kF) % kCells, s = id / (kF * kCells);
  const float* Lf = w.L + (size_t)f * 3 * kC;
  float acc = w.l[f];
  for (int k = 0; k < kC; ++k) acc = fmaf(Lf[k], d4[((size_t)s * kC + k) * kCells + cell], acc);
  for (int k = 0; k < 2 * kC; ++k) acc = fmaf(Lf[kC + k], glob[(size_t)s * 2 * kC + k], acc);
  emb[id] = acc;
}

// Per shape: the cell size s = (hi - lo) / 6 per axis and the margin
// sqrt((s0^2 + s1^2) + s2^2) / 2, float64 (cell centres lo + (i + 1/2) s are
// formed from these where they are used).
__global__ __launch_bounds__(64) void consts_kernel(const Shape* shapes, int n_shapes, double* consts) {
#pragma clang fp contract(off)
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= n_shapes) return;
  const Shape sh = shapes[s];
  double step[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) step[a] = ((double)sh.hi[a] - (double)sh.lo[a]) / (double)kM;
  double* c = consts + (size_t)s * 4;
  c[0] = step[0];
  c[1] = step[1];
  c[2] = step[2];
  c[3] = __builtin_sqrt((step[0] * step[0] + step[1] * step[1]) + step[2] * step[2]) * 0.5;
}

// ------------------------------------------------------------------ pairs --

// Cell selection and mean embeddings: one wave per pair (grid P).  The
// pair's validation, canonical order and float64 relative pose are
// wave-uniform; both objects' cell tests and embedding loads are then issued
// together, and each object's predictor input row [mean (16), pose in the
// other object's frame (12)] goes to the workspace.
__global__ __launch_bounds__(64) void select_kernel(PairArgs A) {
  const int q = blockIdx.x, lane = threadIdx.x;
  if (q >= A.n_pairs) return;
  float* zrow = A.z + (size_t)q * 2 * kIn;
  const int i = A.pairs[2 * q], j = A.pairs[2 * q + 1];
  bool valid = i >= 0 && i < A.n_objs && j >= 0 && j < A.n_objs && i != j;
  const int swp = i > j;
  locc_object oa{}, ob{};
  if (valid) {
    oa = A.objs[swp ? j : i];
    ob = A.objs[swp ? i : j];
    valid = oa.shape >= 0 && oa.shape < A.n_shapes && ob.shape >= 0 && ob.shape < A.n_shapes;
  }
  if (!valid) {  // uniform
    const float nan = __builtin_nanf("");
    if (lane < 2 * kIn / 4) reinterpret_cast<float4*>(zrow)[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (A.pooled && lane < 2 * kF) A.pooled[(size_t)q * 2 * kF + lane] = nan;
    if (lane == 0) {
      A.out[2 * q] = nan;
      A.out[2 * q + 1] = nan;
      if (A.counts) {
        A.counts[2 * q] = -1;
        A.counts[2 * q + 1] = -1;
      }
      A.valid[q] = 0;
      atomicAdd(A.err, 1ull);
    }
    return;
  }
  // float64 relative pose of b in a's frame (the same in every lane)
  double R[9], tt[3];
  {
#pragma clang fp contract(off)
    double Ra[9], Rb[9];
    geo_quat_to_rot(oa.q, Ra);
    geo_quat_to_rot(ob.q, Rb);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) R[3 * r + c] = (Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c]) + Ra[6 + r] * Rb[6 + c];
    const double d0 = (double)ob.p[0] - (double)oa.p[0];
    const double d1 = (double)ob.p[1] - (double)oa.p[1];
    const double d2 = (double)ob.p[2] - (double)oa.p[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) tt[r] = (Ra[r] * d0 + Ra[3 + r] * d1) + Ra[6 + r] * d2;
  }
  const Shape box_a = A.shapes[oa.shape], box_b = A.shapes[ob.shape];
  unsigned long long m[2][4];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double* kc = A.consts + (size_t)(side ? ob.shape : oa.shape) * 4;
    const double step[3] = {kc[0], kc[1], kc[2]}, e = kc[3];
    double own_lo[3], lo_w[3], hi_w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      own_lo[k] = side ? box_b.lo[k] : box_a.lo[k];
      lo_w[k] = (double)(side ? box_a.lo[k] : box_b.lo[k]) - e;
      hi_w[k] = (double)(side ? box_a.hi[k] : box_b.hi[k]) + e;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 64 * r + lane;
      bool in = false;
      if (k < kCells) {
#pragma clang fp contract(off)
        const int ci[3] = {k / (kM * kM), (k / kM) % kM, k % kM};
        double c[3], x[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] = own_lo[a] + ((double)ci[a] + 0.5) * step[a];
        if (side == 0) {  // a's cell into b's frame: R^T (c - t)
          const double e0 = c[0] - tt[0], e1 = c[1] - tt[1], e2 = c[2] - tt[2];
#pragma unroll
          for (int a = 0; a < 3; ++a) x[a] = (R[a] * e0 + R[3 + a] * e1) + R[6 + a] * e2;
        } else {          // b's cell into a's frame: R c + t
#pragma unroll
          for (int a = 0; a < 3; ++a) x[a] = ((R[3 * a] * c[0] + R[3 * a + 1] * c[1]) + R[3 * a + 2] * c[2]) + tt[a];
        }
        in = (x[0] >= lo_w[0]) & (x[0] <= hi_w[0]) & (x[1] >= lo_w[1]) & (x[1] <= hi_w[1]) & (x[2] >= lo_w[2]) &
             (x[2] <= hi_w[2]);
      }
      m[side][r] = __ballot(in);
    }
  }
  // lane = 4 features (f4) x cell residue g mod 16: float4 loads of the selected cells of both
  // objects, issued together, then sums over the 16 residues by shuffles
  const int f4 = lane & 3, g = lane >> 2;
  float4 acc[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const float4* E = reinterpret_cast<const float4*>(A.emb + (size_t)(side ? ob.shape : oa.shape) * kCells * kF) + f4;
    acc[side] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int it = 0; it < (kCells + 15) / 16; ++it) {
      const int k = 16 * it + g;  // 16 consecutive cells per step: one ballot word, m[side][it / 4]
      if (k < kCells && ((m[side][it >> 2] >> (k & 63)) & 1ull)) {
        const float4 v = E[k * (kF / 4)];
        acc[side].x += v.x;
        acc[side].y += v.y;
        acc[side].z += v.z;
        acc[side].w += v.w;
      }
    }
  }
#pragma unroll
  for (int side = 0; side < 2; ++side)
#pragma unroll
    for (int d = 4; d < 64; d <<= 1) {
      acc[side].x += __shfl_xor(acc[side].x, d, 64);
      acc[side].y += __shfl_xor(acc[side].y, d, 64);
      acc[side].z += __shfl_xor(acc[side].z, d, 64);
      acc[side].w += __shfl_xor(acc[side].w, d, 64);
    }
  const int count_a = (int)(__popcll(m[0][0]) + __popcll(m[0][1]) + __popcll(m[0][2]) + __popcll(m[0][3]));
  const int count_b = (int)(__popcll(m[1][0]) + __popcll(m[1][1]) + __popcll(m[1][2]) + __popcll(m[1][3]));
  // lanes 0..3 / 4..7: the means of a / b (4 features each)
  const int side = (lane >> 2) & 1;
  if (lane < 8) {
    const float4 sum = side ? acc[1] : acc[0];
    const int cnt = side ? count_b : count_a;
    const float inv = cnt > 0 ? 1.f / (float)cnt : 0.f;
    const float mean[4] = {sum.x * inv, sum.y * inv, sum.z * inv, sum.w * inv};
    const int f0 = 4 * (lane & 3), cpos = side ^ swp;  // the object's position in the caller's pair
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      zrow[side * kIn + f0 + f] = mean[f];
      if (A.pooled) A.pooled[((size_t)q * 2 + cpos) * kF + f0 + f] = mean[f];
    }
  }
  // the poses, written by one lane each with fixed indices: a in b's frame (-R^T t, R^T), b in
  // a's frame (t, R)
  if (lane == 8) {
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 3; ++a) zrow[kF + a] = (float)(-((R[a] * tt[0] + R[3 + a] * tt[1]) + R[6 + a] * tt[2]));
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) zrow[kF + 3 + 3 * r + c] = (float)R[3 * c + r];
  } else if (lane == 9) {
#pragma unroll
    for (int a = 0; a < 3; ++a) zrow[kIn + kF + a] = (float)tt[a];
#pragma unroll
    for (int a = 0; a < 9; ++a) zrow[kIn + kF + 3 + a] = (float)R[a];
  }
  if (lane == 0) {
    if (A.counts) {
      A.counts[(size_t)q * 2 + swp] = count_a;
      A.counts[(size_t)q * 2 + (swp ^ 1)] = count_b;
    }
    A.valid[q] = 1;
  }
}

constexpr int kTP = 32;                  // pairs per workgroup of the predictor
constexpr int kWaves = 8;                // waves per workgroup, one 16-column stripe each
constexpr int kThreads = 64 * kWaves;
constexpr int kZS = 36;                  // LDS row strides (floats): the inputs padded to 32 columns,
constexpr int kHS = kHP + 4;             // +4 so that 8 consecutive rows start in different banks

struct MlpShared {
  int valid[kTP];
  alignas(16) float Z[2 * kTP][kZS];
  alignas(16) float H[2 * kTP][kHS];     // activations, overwritten layer by layer
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One layer, Out = ReLU(In W^T + b), over RT row tiles of 16 rows, for this
// wave's 16 output columns c0.. (v_mfma_f32_16x16x4f32).  The reduction index
// is permuted so that each lane reads four consecutive inputs at once: at
// k-step 4u + v, lane group g = lane / 16 holds k = 16u + 4g + v, in A (the
// rows, from LDS) and in B (the weight row W[c0 + lane % 16][...], from L2)
// alike.  K16 = K / 16 rounded up; inputs past K are zero in both.
template <int RT, int K, int K16, int IS>
__device__ __forceinline__ void mfma_layer(const float* In, float* Out, const float* __restrict__ W,
                                           const float* __restrict__ bias, int c0, int lane) {
  const int j = lane & 15, g = lane >> 4;
  float4 b[K16];
#pragma unroll
  for (int u = 0; u < K16; ++u) {
    const int k = 16 * u + 4 * g;
    b[u] = k < K ? *reinterpret_cast<const float4*>(W + (size_t)(c0 + j) * K + k) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const float bj = bias[c0 + j];
  f32x4 acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{bj, bj, bj, bj};
#pragma unroll
  for (int u = 0; u < K16; ++u) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float4 a = *reinterpret_cast<const float4*>(In + (rt * 16 + j) * IS + 16 * u + 4 * g);
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[u].x, acc[rt], 0, 0, 0);
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[u].y, acc[rt], 0, 0, 0);
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b[u].z, acc[rt], 0, 0, 0);
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b[u].w, acc[rt], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read In (Out may be the same buffer)
  // D[i][j]: row 4 g + r of the tile, column j
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) Out[(rt * 16 + 4 * g + r) * kHS + c0 + j] = relu(acc[rt][r]);
  __syncthreads();
}

// Predictor MLPs: 32 pairs per workgroup; the 64 object rows come from the workspace.
__global__ __launch_bounds__(kThreads) void mlp_kernel(PairArgs A) {
  __shared__ MlpShared S;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int q0 = blockIdx.x * kTP;
  const int n = A.n_pairs - q0 < kTP ? A.n_pairs - q0 : kTP;  // pairs of this workgroup
  if (t < kTP) S.valid[t] = t < n ? A.valid[q0 + t] : 0;
  for (int id = t; id < 2 * kTP * 8; id += kThreads) {  // 64 rows x 8 float4 (28 inputs, zero to 32)
    const int row = id >> 3, c4 = id & 7;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < 2 * n && c4 < kIn / 4) v = *reinterpret_cast<const float4*>(A.z + ((size_t)q0 * 2 + row) * kIn + 4 * c4);
    *reinterpret_cast<float4*>(&S.Z[row][4 * c4]) = v;
  }
  __syncthreads();
  const int c0 = 16 * wave;
  const float* H = &S.H[0][0];
  float* Hw = &S.H[0][0];
  mfma_layer<4, kIn, 2, kZS>(&S.Z[0][0], Hw, A.w.A[0], A.w.a[0], c0, lane);
  mfma_layer<4, kHP, kHP / 16, kHS>(H, Hw, A.w.A[1], A.w.a[1], c0, lane);
  mfma_layer<4, kHP, kHP / 16, kHS>(H, Hw, A.w.A[2], A.w.a[2], c0, lane);
  {  // max over the two objects of each pair: rows 2q, 2q + 1 -> row q
    float mx[kTP * kHP / kThreads];
#pragma unroll
    for (int r = 0; r < kTP * kHP / kThreads; ++r) {
      const int id = t + r * kThreads, q = id / kHP, c = id % kHP;
      const float u = S.H[2 * q][c], v = S.H[2 * q + 1][c];
      mx[r] = u > v ? u : v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTP * kHP / kThreads; ++r) {
      const int id = t + r * kThreads;
      S.H[id / kHP][id % kHP] = mx[r];
    }
    __syncthreads();
  }
  mfma_layer<2, kHP, kHP / 16, kHS>(H, Hw, A.w.Bw[0], A.w.b[0], c0, lane);
  mfma_layer<2, kHP, kHP / 16, kHS>(H, Hw, A.w.Bw[1], A.w.b[1], c0, lane);
  mfma_layer<2, kHP, kHP / 16, kHS>(H, Hw, A.w.Bw[2], A.w.b[2], c0, lane);
  // output layer and sigmoid: a wave per kTP / kWaves pairs
  const float w_lo = A.w.B4[lane], w_hi = A.w.B4[lane + 64], b4 = A.w.b[3][0];
#pragma unroll
  for (int k = 0; k < kTP / kWaves; ++k) {
    const int q = wave * (kTP / kWaves) + k;
    float v = fmaf(w_lo, S.H[q][lane], w_hi * S.H[q][lane + 64]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0 && S.valid[q]) {
      const float logit = v + b4;
      A.out[2 * (q0 + q)] = logit;
      A.out[2 * (q0 + q) + 1] = 1.f / (1.f + expf(-logit));
    }
  }
}

}  // namespace

// ------------------------------------------------------------------- host --

namespace {

// Floats of each array of the flat weight vector, in order (W, bias per layer).
constexpr size_t kSizes[] = {
    kH * 3, kH, kH * kH, kH, kH * kH, kH,                                  // point MLP
    (size_t)kC * kH * 27, kC, (size_t)kC * kC * 27, kC, (size_t)kC * kC * 27, kC, (size_t)kC * kC * 27, kC,
    (size_t)kC * kC * 27, kC, (size_t)kC * 2 * kC * 27, kC, (size_t)kC * 2 * kC * 27, kC,
    (size_t)kC * 2 * kC * 27, kC,                                          // U-Net
    (size_t)kF * 3 * kC, kF,                                               // embedding map
    (size_t)kHP * kIn, kHP, (size_t)kHP * kHP, kHP, (size_t)kHP * kHP, kHP,  // per-object MLP
    (size_t)kHP * kHP, kHP, (size_t)kHP * kHP, kHP, (size_t)kHP * kHP, kHP, kHP, 1,  // pair MLP, output
};
constexpr int kArrays = sizeof(kSizes) / sizeof(kSizes[0]);

constexpr size_t total_weights() {
  size_t n = 0;
  for (size_t v : kSizes) n += v;
  return n;
}
static_assert(total_weights() == kWeightCount, "weight count");

void offsets(size_t* off) {
  size_t o = 0;
  for (int i = 0; i < kArrays; ++i) {
    off[i] = o;
    o += kSizes[i];
  }
}

// [rows][cols] -> [cols][rows]
void transpose(const float* src, int rows, int cols, float* dst) {
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) dst[(size_t)c * rows + r] = src[(size_t)r * cols + c];
}

// Packed buffer: P2t, P3t, then the U-Net weights transposed to [27][in][out]:
// C[0..3], D[0..3] (input channels 256, 128, 128, 128, 128, 256, 256, 256).
constexpr int kConvIn[8] = {kH, kC, kC, kC, kC, 2 * kC, 2 * kC, 2 * kC};
constexpr size_t kPackSizes[] = {kH * kH, kH * kH,
                                 (size_t)27 * kH * kC, (size_t)27 * kC * kC, (size_t)27 * kC * kC,
                                 (size_t)27 * kC * kC, (size_t)27 * kC * kC, (size_t)27 * 2 * kC * kC,
                                 (size_t)27 * 2 * kC * kC, (size_t)27 * 2 * kC * kC};

// [O][C][27] -> [27][C][O]
void conv_transpose(const float* src, int C, float* dst) {
  for (int o = 0; o < kC; ++o)
    for (int c = 0; c < C; ++c)
      for (int u = 0; u < 27; ++u) dst[((size_t)u * C + c) * kC + o] = src[((size_t)o * C + c) * 27 + u];
}

}  // namespace

size_t packed_floats() {
  size_t n = 0;
  for (size_t v : kPackSizes) n += v;
  return n;
}

void pack_transposed(const float* flat, float* dst) {
  size_t off[kArrays];
  offsets(off);
  float* d = dst;
  transpose(flat + off[2], kH, kH, d);                 // P2
  d += kH * kH;
  transpose(flat + off[4], kH, kH, d);                 // P3
  d += kH * kH;
  for (int i = 0; i < 8; ++i) {                        // U-Net, in the order of kConvIn
    const size_t o = i < 4 ? off[6 + 2 * i] : off[14 + 2 * (i - 4)];
    conv_transpose(flat + o, kConvIn[i], d);
    d += (size_t)27 * kConvIn[i] * kC;
  }
}

PackedNet packed_view(const float* raw, const float* packed) {
  size_t off[kArrays];
  offsets(off);
  PackedNet w{};
  w.P1 = raw + off[0];
  w.p1 = raw + off[1];
  w.p2 = raw + off[3];
  w.p3 = raw + off[5];
  for (int i = 0; i < 4; ++i) {
    w.k[i] = raw + off[7 + 2 * i];
    w.e[i] = raw + off[15 + 2 * i];
  }
  w.L = raw + off[22];
  w.l = raw + off[23];
  for (int i = 0; i < 3; ++i) {
    w.a[i] = raw + off[25 + 2 * i];
    w.b[i] = raw + off[31 + 2 * i];
  }
  w.B4 = raw + off[36];
  w.b[3] = raw + off[37];
  const float* d = packed;
  w.P2t = d;
  d += kH * kH;
  w.P3t = d;
  d += kH * kH;
  for (int i = 0; i < 8; ++i) {
    (i < 4 ? w.C[i] : w.D[i - 4]) = d;
    d += (size_t)27 * kConvIn[i] * kC;
  }
  for (int i = 0; i < 3; ++i) {
    w.A[i] = raw + off[24 + 2 * i];
    w.Bw[i] = raw + off[30 + 2 * i];
  }
  return w;
}

size_t encoder_scratch_floats(int n_shapes, int64_t n_points) {
  const size_t S = (size_t)n_shapes, P = (size_t)n_points;
  return P + (P + 3) / 4 + S * kH * kCells + 7 * S * kC * kB + S * kC * kCells + S * 2 * kC;
}

EncoderBuffers encoder_carve(float* base, int n_shapes, int64_t n_points) {
  const size_t S = (size_t)n_shapes, P = (size_t)n_points;
  EncoderBuffers b{};
  float* p = base;
  b.order = reinterpret_cast<int32_t*>(p);
  p += P;
  b.cell = reinterpret_cast<uint8_t*>(p);
  p += (P + 3) / 4;
  b.grid = p;
  p += S * kH * kCells;
  for (int i = 0; i < 4; ++i) {
    b.c[i] = p;
    p += S * kC * kB;
  }
  for (int i = 0; i < 3; ++i) {
    b.d[i] = p;
    p += S * kC * kB;
  }
  b.d4 = p;
  p += S * kC * kCells;
  b.glob = p;
  return b;
}

namespace {

hipError_t conv(const float* in1, int c1, const float* in2, int c2, const float* Wt, const float* bias, float* out,
                int D, int Do, int pad, int transposed, int n_shapes, hipStream_t s) {
  static_assert(kC % 32 == 0, "output channels in tiles of 32");
  const int C = c1 + c2;
  // eight waves of C / 8 channels each, every wave's channels from one input
  if (C % 16 != 0 || c1 % (C / 8) != 0) return hipErrorInvalidValue;
  ConvArgs a{in1, c1, in2, c2, Wt, bias, out, kC, D, Do, pad, transposed, n_shapes};
  const int N = n_shapes * Do * Do * Do;
  const dim3 grid((unsigned)((N + 31) / 32), kC / 32), block(64 * kConvWaves);
  switch (C / 16) {
    case 8: kernel_launch(conv_kernel<8>, grid, block, 0, s, a); break;
    case 16: kernel_launch(conv_kernel<16>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_encoder(const PackedNet& w, const Shape* shapes, int n_shapes, int max_points, const float* xyz,
                          int64_t n_points, const EncoderBuffers& b, float* emb, double* consts, hipStream_t s) {
  if (n_shapes <= 0 || max_points <= 0) return hipErrorInvalidValue;
  kernel_launch(cell_sort_kernel, dim3(n_shapes), dim3(1024), 0, s, shapes, xyz, n_points, b.order, b.cell);
  kernel_launch(point_mlp_kernel, dim3((max_points + kPts - 1) / kPts, n_shapes), dim3(256), 0, s, w, shapes,
                xyz, n_points, b.order, b.cell, b.grid);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = conv(b.grid, kH, nullptr, 0, w.C[0], w.k[0], b.c[0], kM, 4, 0, 0, n_shapes, s);
  for (int i = 1; i < 4 && e == hipSuccess; ++i)
    e = conv(b.c[i - 1], kC, nullptr, 0, w.C[i], w.k[i], b.c[i], 4, 4, 1, 0, n_shapes, s);
  if (e == hipSuccess) {
    kernel_launch(global_kernel, dim3(n_shapes), dim3(kC), 0, s, b.c[3], b.glob);
    e = hipGetLastError();
  }
  // transposed convs: on the bottleneck, then on [previous, matching conv output]
  if (e == hipSuccess) e = conv(b.c[3], kC, nullptr, 0, w.D[0], w.e[0], b.d[0], 4, 4, 1, 1, n_shapes, s);
  if (e == hipSuccess) e = conv(b.d[0], kC, b.c[2], kC, w.D[1], w.e[1], b.d[1], 4, 4, 1, 1, n_shapes, s);
  if (e == hipSuccess) e = conv(b.d[1], kC, b.c[1], kC, w.D[2], w.e[2], b.d[2], 4, 4, 1, 1, n_shapes, s);
  if (e == hipSuccess) e = conv(b.d[2], kC, b.c[0], kC, w.D[3], w.e[3], b.d4, 4, kM, 0, 1, n_shapes, s);
  if (e == hipSuccess) {
    const int n = n_shapes * kCells * kF;
    kernel_launch(embed_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, b.d4, b.glob, emb, n_shapes);
    kernel_launch(consts_kernel, dim3((n_shapes + 63) / 64), dim3(64), 0, s, shapes, n_shapes, consts);
    e = hipGetLastError();
  }
  return e;
}

size_t pair_workspace_bytes(int n_pairs) {
  const size_t P = (size_t)n_pairs;
  return ((P * 2 * kIn * sizeof(float) + 255) & ~size_t(255)) + P * sizeof(int32_t);
}

void pair_workspace_carve(void* base, int n_pairs, PairArgs& a) {
  const size_t P = (size_t)n_pairs;
  a.z = static_cast<float*>(base);
  a.valid = reinterpret_cast<int32_t*>(static_cast<char*>(base) + ((P * 2 * kIn * sizeof(float) + 255) & ~size_t(255)));
}

hipError_t launch_pairs(const PairArgs& a, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (!a.z || !a.valid) return hipErrorInvalidValue;
  kernel_launch(select_kernel, dim3(a.n_pairs), dim3(64), 0, s, a);
  kernel_launch(mlp_kernel, dim3((a.n_pairs + kTP - 1) / kTP), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace vox
}  // namespace locc
