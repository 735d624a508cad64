// Learned initial guess for the Poisson solve: a 4-layer 3x3x3 convolutional
// network (2 -> 32 -> 32 -> 32 -> 1 channels, ReLU after the first three
// layers, the input's previous-pressure channel added to the output, FP32
// weights and accumulation) on the structured grid of a
// Cartesian base (nx x ny cells, cell j*nx + i) extruded into nz planes.
// Padding is periodic in x and z and replicates the edge cell in y (zero
// gradient at the walls).
//
// Activations are stored [sample][channel][z][y][x] (x fastest).  The
// parameters of layer l are its weights [co][ci][tap], tap = (dz*3 + dy)*3 +
// dx reading the input at (z + dz - 1, y + dy - 1, x + dx - 1), then its
// biases [co]; layers follow each other in one array.  Weight gradients are
// per-block partials summed in a fixed order, so training is deterministic.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"

struct fvx_net {
    int nx = 0, ny = 0, nz = 0, batch = 0, cells = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    float *act[5] = {};   // act[0]: input (2 ch), act[1..3]: 32 ch after ReLU, act[4]: output (1 ch)
    float *g0 = nullptr, *g1 = nullptr;  // gradient ping-pong buffers (32 ch)
    float *part = nullptr;               // weight-gradient partials
    float *lossp = nullptr;              // loss partials
    double *scal = nullptr;              // [0] mean of b removed, [1] scale s
    int step = 0;                        // Adam steps taken
};

namespace fvx {
namespace net {

constexpr int kC = 32;
constexpr int kTaps = 27;
constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {2, kC, kC, kC};
constexpr int kCout[kLayers] = {kC, kC, kC, 1};
constexpr int kBlock = 256;
constexpr int kChunk = 8;        // channels of weights staged in LDS at a time
constexpr int kPosBlocks = 256;  // position ranges of the weight-gradient reduction (32 -> 32 layers)
constexpr int kMaxPosBlocks = 2048;  // ... and at most, for the smaller layers
constexpr int kTile = 64;        // positions staged per pass of the weight gradient
constexpr int kLossBlocks = 256;

constexpr int64_t w_size(int l) { return int64_t(kCout[l]) * kCin[l] * kTaps; }
constexpr int64_t layer_offset(int l) { return l == 0 ? 0 : layer_offset(l - 1) + w_size(l - 1) + kCout[l - 1]; }
constexpr int64_t n_params() { return layer_offset(kLayers); }
constexpr int64_t part_floats() { return int64_t(kPosBlocks) * (int64_t(kC) * kTaps * kC + kC); }

struct Grid {
    int X, Y, Z, cells;
};

// Offsets of the three input neighbours along each axis of cell (x, y, z).
struct Taps {
    int x[3], y[3], z[3];
};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ Taps fwd_taps(const Grid &g, int x, int y, int z) {
    Taps t;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t.x[d] = wrap(x + d - 1, g.X);
        t.y[d] = min(max(y + d - 1, 0), g.Y - 1) * g.X;
        t.z[d] = wrap(z + d - 1, g.Z) * g.X * g.Y;
    }
    return t;
}

// Output cells o that read input cell (x, y, z) through tap offset d along
// each axis: one in x and z (periodic); in y the row y - d + 1 when it
// exists (ya) plus, at the walls, the row whose clamped read lands on y (yb).
struct AdjTaps {
    int x[3], z[3], ya[3], yb[3];
};

__device__ __forceinline__ AdjTaps adj_taps(const Grid &g, int x, int y, int z) {
    AdjTaps t;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        t.x[d] = wrap(x - d + 1, g.X);
        t.z[d] = wrap(z - d + 1, g.Z) * g.X * g.Y;
        const int oy = y - d + 1;
        t.ya[d] = (oy >= 0 && oy < g.Y) ? oy * g.X : -1;
        t.yb[d] = -1;
    }
    if (y == 0) t.yb[0] = 0;                      // o_y = 0 reads row -1, clamped to 0
    if (y == g.Y - 1) t.yb[2] = (g.Y - 1) * g.X;  // o_y = Y-1 reads row Y, clamped to Y-1
    return t;
}

// Position (sample n, cell) of flat index pos < ns*cells and its coordinates.
struct Pos {
    int n, cell, x, y, z;
};

__device__ __forceinline__ Pos pos_of(const Grid &g, int pos) {
    Pos p;
    p.n = pos / g.cells;
    p.cell = pos - p.n * g.cells;
    const int xy = g.X * g.Y;
    p.z = p.cell / xy;
    const int r = p.cell - p.z * xy;
    p.y = r / g.X;
    p.x = r - p.y * g.X;
    return p;
}

// out[n][co][cell] = bias[co] + sum_{ci,tap} W[co][ci][tap] in[n][ci][src(cell, tap)],
// optionally through a ReLU, plus skip[n * skip_stride + cell] when skip is
// given (the output layer adds the network input's previous-pressure
// channel).  Each thread computes all CO outputs of CPT
// cells spaced `per` apart; the weights of kChunk input channels at a time
// are staged in LDS as [ci][tap][co] and read as wave-wide broadcasts.
template <int CO, int CPT>
__global__ __launch_bounds__(kBlock) void k_conv_fwd(Grid g, int ns, int CI, const float *__restrict__ in,
                                                     const float *__restrict__ W, const float *__restrict__ bias,
                                                     float *__restrict__ out, int relu,
                                                     const float *__restrict__ skip, int skip_stride) {
    __shared__ __align__(16) float w_s[kChunk * kTaps * CO];
    const int total = g.cells * ns;
    const int per = (total + CPT - 1) / CPT;
    const int gid = int(blockIdx.x) * blockDim.x + threadIdx.x;
    int base[CPT], obase[CPT], sidx[CPT];
    bool live[CPT];
    Taps t[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int pos = gid + c * per;
        live[c] = gid < per && pos < total;
        const Pos p = pos_of(g, live[c] ? pos : 0);
        t[c] = fwd_taps(g, p.x, p.y, p.z);
        base[c] = p.n * CI * g.cells;
        obase[c] = p.n * CO * g.cells + p.cell;
        sidx[c] = p.n * skip_stride + p.cell;
    }
    float acc[CPT][CO];
#pragma unroll
    for (int co = 0; co < CO; ++co)
#pragma unroll
        for (int c = 0; c < CPT; ++c) acc[c][co] = bias[co];
    for (int c0 = 0; c0 < CI; c0 += kChunk) {
        const int nc = min(kChunk, CI - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < nc * kTaps * CO; i += blockDim.x) {
            const int co = i % CO, rest = i / CO, tap = rest % kTaps, ci = rest / kTaps;
            w_s[i] = W[(co * CI + c0 + ci) * kTaps + tap];
        }
        __syncthreads();
        for (int ci = 0; ci < nc; ++ci) {
            const int coff = (c0 + ci) * g.cells;
#pragma unroll
            for (int tap = 0; tap < kTaps; ++tap) {
                const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
                float a[CPT];
#pragma unroll
                for (int c = 0; c < CPT; ++c) a[c] = in[base[c] + coff + t[c].z[dz] + t[c].y[dy] + t[c].x[dx]];
                const float *w = w_s + (ci * kTaps + tap) * CO;
#pragma unroll
                for (int co = 0; co < CO; ++co)
#pragma unroll
                    for (int c = 0; c < CPT; ++c) acc[c][co] += w[co] * a[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (!live[c]) continue;
#pragma unroll
        for (int co = 0; co < CO; ++co) {
            float v = relu ? fmaxf(acc[c][co], 0.0f) : acc[c][co];
            if (skip) v += skip[sidx[c]];
            out[obase[c] + co * g.cells] = v;
        }
    }
}

// The output layer (32 -> 1 channel): out[n][cell] = bias + sum_{ci,tap}
// W[ci][tap] in[n][ci][src(cell, tap)] + skip.  A dot product per cell (no
// matrix-core shape fits M = 1), so on the vector ALU with the input channels
// split over kSplit1 lanes per cell (each lane 32 / kSplit1 channels, all 27
// taps), the lanes' sums added by two xor shuffles: four times the threads of
// one lane per cell, which a single-sample inference needs to fill the GPU.
constexpr int kSplit1 = 4;
// From this many cells (four single-sample 64 x 64 x 8 grids) on, the output
// layer takes four cells per thread instead (k_conv_fwd<1, 4>): on the 16-sample
// training batch 163 us against 230 us split; one sample 107 us against 29 us.
constexpr int64_t kFwd1Split = int64_t(1) << 17;

__global__ __launch_bounds__(kBlock) void k_conv_fwd1(Grid g, int ns, const float *__restrict__ in,
                                                      const float *__restrict__ W, const float *__restrict__ bias,
                                                      float *__restrict__ out, const float *__restrict__ skip,
                                                      int skip_stride) {
    constexpr int CI = kC, CG = CI / kSplit1;
    __shared__ float w_s[CI * kTaps];  // [ci][tap]
    for (int i = threadIdx.x; i < CI * kTaps; i += blockDim.x) w_s[i] = W[i];
    __syncthreads();
    const int total = g.cells * ns;
    const int gid = int(blockIdx.x) * blockDim.x + threadIdx.x;
    const int pos = gid / kSplit1, part = gid % kSplit1;  // kSplit1 consecutive lanes share a cell
    const bool live = pos < total;
    const Pos p = pos_of(g, live ? pos : 0);
    const Taps t = fwd_taps(g, p.x, p.y, p.z);
    const float *src = in + (int64_t(p.n) * CI + part * CG) * g.cells;
    const float *w = w_s + part * CG * kTaps;
    float acc = 0.0f;
    for (int ci = 0; ci < CG; ++ci) {
#pragma unroll
        for (int tap = 0; tap < kTaps; ++tap)
            acc += w[ci * kTaps + tap] * src[int64_t(ci) * g.cells + t.z[tap / 9] + t.y[(tap / 3) % 3] + t.x[tap % 3]];
    }
    acc += __shfl_xor(acc, 1, kSplit1);
    acc += __shfl_xor(acc, 2, kSplit1);
    if (live && part == 0) {
        float v = bias[0] + acc;
        if (skip) v += skip[p.n * skip_stride + p.cell];
        out[int64_t(p.n) * g.cells + p.cell] = v;
    }
}

typedef float mfma_acc16 __attribute__((ext_vector_type(16)));

// The 32-output-channel layers as an implicit GEMM on the matrix cores
// (v_mfma_f32_32x32x2_f32, FP32 in and out):
//   D[co][cell] = bias[co] + sum_{tap, ci} W[co][ci][tap] in[ci][src(cell, tap)]
// with M = 32 output channels, N = 32 cells per MFMA column block (NB blocks
// per wave) and K = 27 * CI taken two input channels at a time.  Operand
// layouts of the 32x32x2 instruction: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; accumulator register r of lane l is
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  The weights of one z-offset of
// the stencil (9 taps) at a time are staged in LDS as [tap][ci][co], so the
// A operand is a conflict-free LDS read; B is a gather of 32 consecutive
// cells per channel.  ReLU on output.
template <int CI, int NB>
__global__ __launch_bounds__(kBlock) void k_conv_fwd_mfma(Grid g, int ns, const float *__restrict__ in,
                                                          const float *__restrict__ W,
                                                          const float *__restrict__ bias, float *__restrict__ out) {
    constexpr int CO = kC;
    __shared__ __align__(16) float w_s[9 * CI * CO];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 31, hi = lane >> 5;
    const int total = g.cells * ns;
    const int first = (int(blockIdx.x) * (kBlock / 64) + wave) * (32 * NB);
    int base[NB], cell[NB], nn[NB];
    bool live[NB];
    Taps t[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int pos = first + 32 * b + lo;
        live[b] = pos < total;
        const Pos p = pos_of(g, live[b] ? pos : 0);
        t[b] = fwd_taps(g, p.x, p.y, p.z);
        base[b] = p.n * CI * g.cells + hi * g.cells;
        cell[b] = p.cell;
        nn[b] = p.n;
    }
    mfma_acc16 acc[NB];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float bv = bias[8 * (r / 4) + 4 * hi + (r % 4)];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b][r] = bv;
    }
#pragma unroll  // constant dz: the tap offsets t[b].z[dz] stay in registers
    for (int dz = 0; dz < 3; ++dz) {
        __syncthreads();
        for (int i = threadIdx.x; i < 9 * CI * CO; i += blockDim.x) {
            const int co = i % CO, rest = i / CO, ci = rest % CI, tl = rest / CI;
            w_s[i] = W[(co * CI + ci) * kTaps + dz * 9 + tl];
        }
        __syncthreads();
#pragma unroll
        for (int tl = 0; tl < 9; ++tl) {
            const int dy = tl / 3, dx = tl % 3;
            int off[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) off[b] = base[b] + t[b].z[dz] + t[b].y[dy] + t[b].x[dx];
#pragma unroll
            for (int c = 0; c < CI; c += 2) {
                const float a = w_s[(tl * CI + c + hi) * CO + lo];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float bx = in[off[b] + c * g.cells];
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bx, acc[b], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!live[b]) continue;
        float *o = out + nn[b] * CO * g.cells + cell[b];
#pragma unroll
        for (int r = 0; r < 16; ++r) o[(8 * (r / 4) + 4 * hi + (r % 4)) * g.cells] = fmaxf(acc[b][r], 0.0f);
    }
}

// Gradient with respect to a 32-channel layer input:
// din[n][ci][p] = sum_{co,tap} W[co][ci][tap] sum_{o reads p at tap} dout[n][co][o],
// multiplied by the ReLU derivative (act_in > 0) of the layer that produced
// the input.  Weights staged as [co][tap][ci].
template <int CPT>
__global__ __launch_bounds__(kBlock) void k_conv_bwd_data(Grid g, int ns, int CO, const float *__restrict__ dout,
                                                          const float *__restrict__ W,
                                                          const float *__restrict__ act_in, float *__restrict__ din) {
    constexpr int CI = kC;
    __shared__ __align__(16) float w_s[kChunk * kTaps * CI];
    const int total = g.cells * ns;
    const int per = (total + CPT - 1) / CPT;
    const int gid = int(blockIdx.x) * blockDim.x + threadIdx.x;
    int dbase[CPT], ibase[CPT];
    bool live[CPT];
    AdjTaps t[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int pos = gid + c * per;
        live[c] = gid < per && pos < total;
        const Pos p = pos_of(g, live[c] ? pos : 0);
        t[c] = adj_taps(g, p.x, p.y, p.z);
        dbase[c] = p.n * CO * g.cells;
        ibase[c] = p.n * CI * g.cells + p.cell;
    }
    float acc[CPT][CI];
#pragma unroll
    for (int ci = 0; ci < CI; ++ci)
#pragma unroll
        for (int c = 0; c < CPT; ++c) acc[c][ci] = 0.0f;
    for (int c0 = 0; c0 < CO; c0 += kChunk) {
        const int nc = min(kChunk, CO - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < nc * kTaps * CI; i += blockDim.x) {
            const int ci = i % CI, rest = i / CI, tap = rest % kTaps, co = rest / kTaps;
            w_s[i] = W[((c0 + co) * CI + ci) * kTaps + tap];
        }
        __syncthreads();
        for (int co = 0; co < nc; ++co) {
            const int coff = (c0 + co) * g.cells;
#pragma unroll
            for (int tap = 0; tap < kTaps; ++tap) {
                const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
                float s[CPT];
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const float *d = dout + dbase[c] + coff + t[c].z[dz] + t[c].x[dx];
                    // Both reads are in bounds (offset 0 stands in for a missing row) and
                    // selected without a branch, which keeps the unrolled taps in registers.
                    const float va = d[max(t[c].ya[dy], 0)], vb = d[max(t[c].yb[dy], 0)];
                    s[c] = (t[c].ya[dy] >= 0 ? va : 0.0f) + (t[c].yb[dy] >= 0 ? vb : 0.0f);
                }
                const float *w = w_s + (co * kTaps + tap) * CI;
#pragma unroll
                for (int ci = 0; ci < CI; ++ci)
#pragma unroll
                    for (int c = 0; c < CPT; ++c) acc[c][ci] += w[ci] * s[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (!live[c]) continue;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const int o = ibase[c] + ci * g.cells;
            din[o] = act_in[o] > 0.0f ? acc[c][ci] : 0.0f;
        }
    }
}

// The same gradient for a 32-channel output gradient on the matrix cores:
//   D[ci][p] = sum_{tap, co} W[co][ci][tap] adj(dout[co])(p, tap)
// M = 32 input channels, N = 32 positions per column block, K = 27 * 32 two
// output channels at a time; operand and accumulator layouts as in
// k_conv_fwd_mfma, weights staged per z-offset as [tap][co][ci].
template <int NB>
__global__ __launch_bounds__(kBlock) void k_conv_bwd_data_mfma(Grid g, int ns, const float *__restrict__ dout,
                                                               const float *__restrict__ W,
                                                               const float *__restrict__ act_in,
                                                               float *__restrict__ din) {
    constexpr int CI = kC, CO = kC;
    __shared__ __align__(16) float w_s[9 * CO * CI];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 31, hi = lane >> 5;
    const int total = g.cells * ns;
    const int first = (int(blockIdx.x) * (kBlock / 64) + wave) * (32 * NB);
    int dbase[NB], ibase[NB];
    bool live[NB];
    AdjTaps t[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int pos = first + 32 * b + lo;
        live[b] = pos < total;
        const Pos p = pos_of(g, live[b] ? pos : 0);
        t[b] = adj_taps(g, p.x, p.y, p.z);
        dbase[b] = p.n * CO * g.cells + hi * g.cells;
        ibase[b] = p.n * CI * g.cells + p.cell;
    }
    mfma_acc16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;
#pragma unroll  // constant dz: the tap offsets t[b].z[dz] stay in registers
    for (int dz = 0; dz < 3; ++dz) {
        __syncthreads();
        for (int i = threadIdx.x; i < 9 * CO * CI; i += blockDim.x) {
            const int ci = i % CI, rest = i / CI, co = rest % CO, tl = rest / CO;
            w_s[i] = W[(co * CI + ci) * kTaps + dz * 9 + tl];
        }
        __syncthreads();
#pragma unroll
        for (int tl = 0; tl < 9; ++tl) {
            const int dy = tl / 3, dx = tl % 3;
            const float *d[NB];
            int ya[NB], yb[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                d[b] = dout + dbase[b] + t[b].z[dz] + t[b].x[dx];
                ya[b] = t[b].ya[dy];
                yb[b] = t[b].yb[dy];
            }
#pragma unroll
            for (int c = 0; c < CO; c += 2) {
                const float a = w_s[(tl * CO + c + hi) * CI + lo];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    // both reads in bounds (offset 0 stands in for a missing row), selected without a branch
                    const float *dc = d[b] + c * g.cells;
                    const float va = dc[max(ya[b], 0)], vb = dc[max(yb[b], 0)];
                    const float bx = (ya[b] >= 0 ? va : 0.0f) + (yb[b] >= 0 ? vb : 0.0f);
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bx, acc[b], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!live[b]) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = ibase[b] + (8 * (r / 4) + 4 * hi + (r % 4)) * g.cells;
            din[o] = act_in[o] > 0.0f ? acc[b][r] : 0.0f;
        }
    }
}

// Weight and bias gradient partials over the positions [p0, p0 + per) of
// block x: thread j of block y owns the (ci, tap) pair y*blockDim + j and
// accumulates sum_pos dout[co][pos] * in[ci][src(pos, tap)] for every co.
// part[bx][(ci*27 + tap)*CO + co]; the biases at part[bx][CI*27*CO + co].
template <int CO>
__global__ __launch_bounds__(kBlock) void k_conv_bwd_w(Grid g, int ns, int CI, const float *__restrict__ dout,
                                                       const float *__restrict__ in, int per,
                                                       float *__restrict__ part) {
    __shared__ __align__(16) float d_s[kTile * CO];  // [j][co]
    __shared__ int p_s[kTile * 4];                    // input base, x, y, z of position j
    const int total = g.cells * ns;
    const int p0 = int(blockIdx.x) * per, p1 = min(total, p0 + per);
    const int npair = CI * kTaps;
    const int pair = int(blockIdx.y) * blockDim.x + threadIdx.x;
    const bool mine = pair < npair;
    const int ci = mine ? pair / kTaps : 0, tap = mine ? pair % kTaps : 0;
    const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
    const bool do_bias = blockIdx.y == 0 && threadIdx.x < CO;
    float acc[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) acc[co] = 0.0f;
    float bacc = 0.0f;
    for (int t0 = p0; t0 < p1; t0 += kTile) {
        const int nt = min(kTile, p1 - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < kTile * CO; i += blockDim.x) {
            const int j = i % kTile, co = i / kTile;
            float v = 0.0f;
            if (j < nt) {
                const Pos p = pos_of(g, t0 + j);
                v = dout[(p.n * CO + co) * g.cells + p.cell];
            }
            d_s[j * CO + co] = v;
        }
        for (int j = threadIdx.x; j < nt; j += blockDim.x) {
            const Pos p = pos_of(g, t0 + j);
            p_s[4 * j] = p.n * CI * g.cells;
            p_s[4 * j + 1] = p.x;
            p_s[4 * j + 2] = p.y;
            p_s[4 * j + 3] = p.z;
        }
        __syncthreads();
        if (mine) {
            const float *src = in + ci * g.cells;
#pragma unroll 8  // eight gathers in flight; each accumulator still sums in position order
            for (int j = 0; j < nt; ++j) {
                const int xs = wrap(p_s[4 * j + 1] + dx - 1, g.X);
                const int ys = min(max(p_s[4 * j + 2] + dy - 1, 0), g.Y - 1);
                const int zs = wrap(p_s[4 * j + 3] + dz - 1, g.Z);
                const float a = src[p_s[4 * j] + (zs * g.Y + ys) * g.X + xs];
                const float *d = d_s + j * CO;
#pragma unroll
                for (int co = 0; co < CO; ++co) acc[co] += d[co] * a;
            }
        }
        if (do_bias)
            for (int j = 0; j < nt; ++j) bacc += d_s[j * CO + threadIdx.x];
    }
    float *out = part + size_t(blockIdx.x) * (size_t(npair) * CO + CO);
    if (mine)
#pragma unroll
        for (int co = 0; co < CO; ++co) out[pair * CO + co] = acc[co];
    if (do_bias) out[npair * CO + threadIdx.x] = bacc;
}

// Weight gradient of a layer with 32 output channels on the matrix cores:
//   dW[co][ci][tap] = sum_pos dout[co][pos] in[ci][src(pos, tap)]
// as a GEMM with M = 32 output channels, N = the (ci, tap) pairs in column
// blocks of 32 and K = the block's positions, two at a time
// (v_mfma_f32_32x32x2_f32; operand and accumulator layouts as in
// k_conv_fwd_mfma).  CI = 32: column block cb is tap cb with ci = column;
// CI < 32: column n of block cb is pair 32 cb + n = ci * 27 + tap.  Per chunk
// of 64 positions the block stages dout as [position][co]; in round q, wave
// w gathers column block 4 q + w of the input as [position][column] (one
// position per lane: coalesced along the positions) and runs 32 MFMAs on it.
// The bias gradient and the partials' layout are those of k_conv_bwd_w, so
// k_fold_w sums them in the same fixed order.
constexpr int kWChunk = 64;
constexpr int kWPad = kC + 1;  // LDS row stride: conflict-free column writes

template <int CI>
__global__ __launch_bounds__(kBlock) void k_conv_bwd_w_mfma(Grid g, int ns, const float *__restrict__ dout,
                                                            const float *__restrict__ in, int per,
                                                            float *__restrict__ part) {
    constexpr int CO = kC, NPAIR = CI * kTaps, NCB = (NPAIR + 31) / 32, ROUNDS = (NCB + 3) / 4;
    __shared__ float d_s[kWChunk * kWPad];     // [k][co]
    __shared__ float a_s[4][kWChunk * kWPad];  // per wave: [k][column]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 31, hi = lane >> 5;
    const int total = g.cells * ns;
    const int p0 = int(blockIdx.x) * per, p1 = min(total, p0 + per);
    float *a_w = a_s[wave];
    mfma_acc16 acc[ROUNDS];
#pragma unroll
    for (int q = 0; q < ROUNDS; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    float bacc = 0.0f;
    for (int c0 = p0; c0 < p1; c0 += kWChunk) {
        const int nt = min(kWChunk, p1 - c0);
        __syncthreads();  // the previous chunk's reads of d_s are done
        for (int i = threadIdx.x; i < kWChunk * CO; i += kBlock) {
            const int k = i % kWChunk, co = i / kWChunk;
            float v = 0.0f;
            if (k < nt) {
                const Pos p = pos_of(g, c0 + k);
                v = dout[(p.n * CO + co) * g.cells + p.cell];
            }
            d_s[k * kWPad + co] = v;
        }
        // this lane's position of the chunk (lane < nt)
        const bool mine = lane < nt;
        const Pos pk = pos_of(g, mine ? c0 + lane : p0);
        const float *in_n = in + int64_t(pk.n) * CI * g.cells;
        auto src_cell = [&](int tap) {
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
            const int xs = wrap(pk.x + dx - 1, g.X);
            const int ys = min(max(pk.y + dy - 1, 0), g.Y - 1);
            const int zs = wrap(pk.z + dz - 1, g.Z);
            return (zs * g.Y + ys) * g.X + xs;
        };
        __syncthreads();
        if (threadIdx.x < CO)
            for (int k = 0; k < nt; ++k) bacc += d_s[k * kWPad + threadIdx.x];
#pragma unroll
        for (int q = 0; q < ROUNDS; ++q) {
            const int cb = 4 * q + wave;  // uniform over the wave
            if (cb < NCB) {
                float v[32];
                if constexpr (CI == 32) {
                    // all 32 loads in flight (staging them in two halves of 16 gave two
                    // waves per SIMD but measured slower: 560 -> 600 us)
                    const float *src = in_n + src_cell(cb);
#pragma unroll
                    for (int n = 0; n < 32; ++n) v[n] = mine ? src[int64_t(n) * g.cells] : 0.0f;
#pragma unroll
                    for (int n = 0; n < 32; ++n) a_w[lane * kWPad + n] = v[n];
                } else {
#pragma unroll
                    for (int n = 0; n < 32; ++n) {
                        const int pr = 32 * cb + n;
                        v[n] = (mine && pr < NPAIR) ? in_n[int64_t(pr / kTaps) * g.cells + src_cell(pr % kTaps)] : 0.0f;
                    }
#pragma unroll
                    for (int n = 0; n < 32; ++n) a_w[lane * kWPad + n] = v[n];
                }
            }
            __syncthreads();  // a_w written (each wave reads only its own)
            if (cb < NCB) {
#pragma unroll
                for (int k0 = 0; k0 < kWChunk; k0 += 2) {
                    const float a = d_s[(k0 + hi) * kWPad + lo];
                    const float b = a_w[(k0 + hi) * kWPad + lo];
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[q], 0, 0, 0);
                }
            }
            __syncthreads();  // a_w read before the next round overwrites it
        }
    }
    float *out = part + size_t(blockIdx.x) * (size_t(NPAIR) * CO + CO);
#pragma unroll
    for (int q = 0; q < ROUNDS; ++q) {
        const int cb = 4 * q + wave;
        const int pr = CI == 32 ? lo * kTaps + cb : 32 * cb + lo;
        if (cb >= NCB || pr >= NPAIR) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) out[pr * CO + 8 * (r / 4) + 4 * hi + (r % 4)] = acc[q][r];
    }
    if (threadIdx.x < CO) out[NPAIR * CO + threadIdx.x] = bacc;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Weight gradient of the output layer (32 -> 1 channel) on the matrix cores,
// with the tap moved from the input onto the output gradient (the adjoint of
// the padding, as in the data gradient):
//   dW[0][ci][tap] = sum_p in[ci][p] adj(dout)(p, tap),
// adj(dout)(p, tap) = the sum of dout over the outputs that read p through
// tap.  M = 32 input channels, N = the 27 taps (padded to 32), K = positions,
// two at a time.  Wave w takes chunks w, w + 4, ... of 64 positions of the
// block's range: each lane stages its position's 32 inputs and 27 adjoint
// taps in LDS as [position][column] and the wave runs 32 MFMAs; the four
// waves' sums are added in wave order.  Partials: part[bx][ci * 27 + tap] and
// the bias gradient (sum of dout) at part[bx][32 * 27].
__global__ __launch_bounds__(kBlock) void k_conv_bwd_w1_mfma(Grid g, int ns, const float *__restrict__ dout,
                                                             const float *__restrict__ in, int per,
                                                             float *__restrict__ part) {
    constexpr int CI = kC;
    __shared__ float i_s[4][kWChunk * kWPad];  // per wave: [k][ci]
    __shared__ float d_s[4][kWChunk * kWPad];  // per wave: [k][tap]
    __shared__ float b_s[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 31, hi = lane >> 5;
    const int total = g.cells * ns;
    const int p0 = int(blockIdx.x) * per, p1 = min(total, p0 + per);
    const int nchunk = (p1 - p0 + kWChunk - 1) / kWChunk;
    float *iw = i_s[wave], *dw = d_s[wave];
    mfma_acc16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    float bsum = 0.0f;
    for (int j0 = 0; j0 < nchunk; j0 += 4) {  // the same trip count in every wave
        const int j = j0 + wave;
        const int c0 = p0 + j * kWChunk;
        const bool live = j < nchunk && c0 + lane < p1;
        const Pos pk = pos_of(g, live ? c0 + lane : p0);
        const float *src = in + int64_t(pk.n) * CI * g.cells + pk.cell;
        const float *dn = dout + int64_t(pk.n) * g.cells;
        const AdjTaps t = adj_taps(g, pk.x, pk.y, pk.z);
        float v[CI], a[kTaps];
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) v[ci] = live ? src[int64_t(ci) * g.cells] : 0.0f;
#pragma unroll
        for (int tap = 0; tap < kTaps; ++tap) {
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
            const int ya = t.ya[dy], yb = t.yb[dy];
            // both reads in bounds (offset 0 stands in for a missing row), selected without a branch
            const float *d = dn + t.z[dz] + t.x[dx];
            const float va = d[max(ya, 0)], vb = d[max(yb, 0)];
            a[tap] = live ? (ya >= 0 ? va : 0.0f) + (yb >= 0 ? vb : 0.0f) : 0.0f;
        }
        bsum += wave_sum_f(live ? dn[pk.cell] : 0.0f);
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) iw[lane * kWPad + ci] = v[ci];
#pragma unroll
        for (int n = 0; n < 32; ++n) dw[lane * kWPad + n] = n < kTaps ? a[n] : 0.0f;
        __syncthreads();
#pragma unroll
        for (int k0 = 0; k0 < kWChunk; k0 += 2) {
            const float x = iw[(k0 + hi) * kWPad + lo];
            const float y = dw[(k0 + hi) * kWPad + lo];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // D[ci][tap]: register r of lane l holds ci = 8 (r / 4) + 4 (l / 32) + r % 4, tap = l % 32
    float *red = &i_s[0][0];  // [wave][r][lane] (4096 floats of the 4 x 2112), reused after the last barrier
#pragma unroll
    for (int r = 0; r < 16; ++r) red[(wave * 16 + r) * 64 + lane] = acc[r];
    if (lane == 0) b_s[wave] = bsum;
    __syncthreads();
    float *out = part + size_t(blockIdx.x) * (size_t(CI) * kTaps + 1);
    if (wave == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float s = 0.0f;
            for (int w = 0; w < 4; ++w) s += red[(w * 16 + r) * 64 + lane];
            if (lo < kTaps) out[(8 * (r / 4) + 4 * hi + (r % 4)) * kTaps + lo] = s;
        }
        if (lane == 0) out[CI * kTaps] = ((b_s[0] + b_s[1]) + b_s[2]) + b_s[3];
    }
}

// Gradients of one layer (weights [co][ci][tap], biases) = sum over the
// position blocks of the partials, in block order.
__global__ __launch_bounds__(kBlock) void k_fold_w(const float *__restrict__ part, int nblk, int CI, int CO,
                                                   float *__restrict__ gw, float *__restrict__ gb) {
    const int npair = CI * kTaps;
    const int stride = npair * CO + CO;
    for (int v = int(blockIdx.x) * blockDim.x + threadIdx.x; v < stride; v += gridDim.x * blockDim.x) {
        float s = 0.0f;
#pragma unroll 8  // loads in flight; the sum keeps block order
        for (int b = 0; b < nblk; ++b) s += part[size_t(b) * stride + v];
        if (v < npair * CO) {
            const int pr = v / CO, co = v % CO;
            gw[(co * CI + pr / kTaps) * kTaps + pr % kTaps] = s;
        } else {
            gb[v - npair * CO] = s;
        }
    }
}

// Mean-squared error over n values: d = 2 (out - t) / n and per-block
// partial sums of (out - t)^2.
__global__ __launch_bounds__(kBlock) void k_mse(const float *__restrict__ out, const float *__restrict__ t, int n,
                                                float *__restrict__ d, float *__restrict__ part) {
    __shared__ float s[kBlock];
    float acc = 0.0f;
    for (int i = int(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float e = out[i] - t[i];
        d[i] = 2.0f * e / float(n);
        acc += e * e;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Adam with bias correction (Kingma and Ba, 2015); c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ __launch_bounds__(kBlock) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                                 float *__restrict__ m, float *__restrict__ v, int n, float lr,
                                                 float b1, float b2, float eps, float c1, float c2) {
    for (int i = int(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(float *__restrict__ p, int n) {
    for (int i = int(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0f;
}

__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Scales of one sample (one block): s[0] = plain mean of b (0 unless the
// operator is singular), s[1] = rms over the cells of the source density
// f = (b - s[0]) / (area * dz), or 1 when it is zero.  B: AoS [n_b][ld].
// Loads in flight per thread in the single-block reductions below: each
// thread issues kBatch loads before it adds any of them (one memory round
// trip per kBatch elements instead of one per element); the sums keep the
// element order of a plain strided loop.
constexpr int kBatch = 8;

// Element i of AoS [n_b][ld] for plane-fastest flat index i = c * k + l,
// stepped by `stride` without a division per element.
struct FlatIdx {
    int c, l, dc, dl, k;
    __device__ FlatIdx(int i, int stride, int kk) : c(i / kk), l(i % kk), dc(stride / kk), dl(stride % kk), k(kk) {}
    __device__ void step() {
        c += dc;
        l += dl;
        if (l >= k) {
            l -= k;
            ++c;
        }
    }
};

__global__ __launch_bounds__(1024) void k_scale(Grid g, const double *__restrict__ B, int ld,
                                                const double *__restrict__ area, double inv_dz, int singular,
                                                double *__restrict__ s) {
    __shared__ double red[1024];
    const int k = g.Z, n = g.cells, T = blockDim.x;
    double a = 0.0;
    {
        FlatIdx ix(threadIdx.x, T, k);
        for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * T) {
            double v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                v[u] = i0 + u * T < n ? B[int64_t(ix.c) * ld + ix.l] : 0.0;
                ix.step();
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) a += v[u];
        }
    }
    const double sum = block_sum(a, red);
    const double mean = singular ? sum / double(n) : 0.0;
    a = 0.0;
    {
        FlatIdx ix(threadIdx.x, T, k);
        for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * T) {
            double v[kBatch], ar[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const bool in = i0 + u * T < n;
                v[u] = in ? B[int64_t(ix.c) * ld + ix.l] : mean;
                ar[u] = in ? area[ix.c] : 1.0;
                ix.step();
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const double f = (v[u] - mean) / ar[u] * inv_dz;
                a += f * f;
            }
        }
    }
    const double rms = sqrt(block_sum(a, red) / double(n));
    if (threadIdx.x == 0) {
        s[0] = mean;
        s[1] = rms > 0.0 ? rms : 1.0;
    }
}

// Network input of one sample: in[0][cell] = f / s, in[1][cell] = p_prev / s
// (0 without a previous pressure); the optional target is x* / s.
__global__ __launch_bounds__(kBlock) void k_prepare(Grid g, const double *__restrict__ B,
                                                    const double *__restrict__ P, const double *__restrict__ Xs, int ld,
                                                    const double *__restrict__ area, double inv_dz,
                                                    const double *__restrict__ s, float *__restrict__ in,
                                                    float *__restrict__ target) {
    const int nb = g.X * g.Y;
    const double mean = s[0], sc = s[1];
    for (int i = int(blockIdx.x) * blockDim.x + threadIdx.x; i < g.cells; i += gridDim.x * blockDim.x) {
        const int c = i % nb, z = i / nb;
        const int o = c * ld + z;
        in[i] = float((B[o] - mean) / area[c] * inv_dz / sc);
        in[g.cells + i] = P ? float(P[o] / sc) : 0.0f;
        if (target) target[i] = float(Xs[o] / sc);
    }
}

// x0 = s * (out - mean(out)) (mean removed only for a singular operator),
// written into the AoS [n_b][ld] vector X.
// Every block sums all of out in the same order (the same mean, bitwise), then
// writes its range of cells, all planes of a cell by one thread (a contiguous
// AoS row): the writes spread over the blocks instead of one CU's scattered stores.
constexpr int kGuessOutBlocks = 32;

__global__ __launch_bounds__(1024) void k_guess_out(Grid g, const float *__restrict__ out,
                                                    const double *__restrict__ s, int singular,
                                                    double *__restrict__ X, int ld) {
    __shared__ double red[1024];
    const int nb = g.X * g.Y, k = g.Z, n = g.cells, T = blockDim.x;
    double a = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * T) {
        float v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) v[u] = i0 + u * T < n ? out[i0 + u * T] : 0.0f;
#pragma unroll
        for (int u = 0; u < kBatch; ++u) a += double(v[u]);
    }
    const double sum = block_sum(a, red);
    const double mean = singular ? sum / double(n) : 0.0;
    const double sc = s[1];
    // out is [plane][cell]; X is AoS [cell][ld]
    for (int c = int(blockIdx.x) * T + threadIdx.x; c < nb; c += int(gridDim.x) * T)
        for (int l = 0; l < k; ++l) X[int64_t(c) * ld + l] = sc * (double(out[int64_t(l) * nb + c]) - mean);
}

Grid grid_of(const fvx_net *n) { return Grid{n->nx, n->ny, n->nz, n->cells}; }

template <int CO, int CPT>
void conv_fwd(const Grid &g, int ns, int CI, const float *in, const float *W, const float *b, float *out, int relu,
              const float *skip, hipStream_t s) {
    const int64_t threads = ceil_div(int64_t(g.cells) * ns, CPT);
    hipLaunchKernelGGL((k_conv_fwd<CO, CPT>), dim3(unsigned(ceil_div(threads, kBlock))), dim3(kBlock), 0, s, g, ns,
                       CI, in, W, b, out, relu, skip, 2 * g.cells);
}

// 32-output-channel layer on the matrix cores: one wave per 32 * NB cells,
// four waves per workgroup; two column blocks per wave once there are
// enough cells for every CU to hold several workgroups.
template <int CI>
void conv_fwd_mfma(const Grid &g, int ns, const float *in, const float *W, const float *b, float *out,
                   hipStream_t s) {
    const int64_t total = int64_t(g.cells) * ns;
    if (total >= int64_t(2048) * 256) {
        const unsigned blocks = unsigned(ceil_div(total, (kBlock / 64) * 64));
        hipLaunchKernelGGL((k_conv_fwd_mfma<CI, 2>), dim3(blocks), dim3(kBlock), 0, s, g, ns, in, W, b, out);
    } else {
        const unsigned blocks = unsigned(ceil_div(total, (kBlock / 64) * 32));
        hipLaunchKernelGGL((k_conv_fwd_mfma<CI, 1>), dim3(blocks), dim3(kBlock), 0, s, g, ns, in, W, b, out);
    }
}

void forward(fvx_net *net, int ns, const float *in, hipStream_t s) {
    const Grid g = grid_of(net);
    const float *src = in;
    for (int l = 0; l < kLayers; ++l) {
        const float *W = net->params + layer_offset(l);
        const float *b = W + w_size(l);
        if (kCout[l] == kC) {
            if (kCin[l] == 2)
                conv_fwd_mfma<2>(g, ns, src, W, b, net->act[l + 1], s);
            else
                conv_fwd_mfma<kC>(g, ns, src, W, b, net->act[l + 1], s);
        } else if (int64_t(g.cells) * ns >= kFwd1Split) {
            // enough cells to fill the GPU with four cells per thread (coalesced along the cells)
            conv_fwd<1, 4>(g, ns, kCin[l], src, W, b, net->act[l + 1], 0, in + g.cells, s);
        } else {
            const int64_t threads = int64_t(g.cells) * ns * kSplit1;
            hipLaunchKernelGGL(k_conv_fwd1, dim3(unsigned(ceil_div(threads, kBlock))), dim3(kBlock), 0, s, g, ns, src,
                               W, b, net->act[l + 1], in + g.cells, 2 * g.cells);
        }
        src = net->act[l + 1];
    }
    FVX_HIP(hipGetLastError());
}

// Forward pass, loss and all parameter gradients (into net->grads); returns
// the mean-squared error after synchronising the stream.
double backward(fvx_net *n, int ns, const float *in, const float *target, hipStream_t s) {
    const Grid g = grid_of(n);
    forward(n, ns, in, s);
    const int nout = g.cells * ns;
    hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kBlock), 0, s, n->act[4], target, nout, n->g0, n->lossp);
    FVX_HIP(hipGetLastError());
    float *dcur = n->g0, *dnext = n->g1;
    const int64_t threads2 = ceil_div(nout, 2);
    for (int l = kLayers - 1; l >= 0; --l) {
        const int CI = kCin[l], CO = kCout[l];
        const float *W = n->params + layer_offset(l);
        float *gw = n->grads + layer_offset(l), *gb = gw + w_size(l);
        const float *lin = l == 0 ? in : n->act[l];
        // Position blocks of the weight-gradient partials: as many as the
        // partial buffer holds for this layer, at most kMaxPosBlocks and at
        // least 64 positions each (short per-thread chains for the small
        // layers; 256 blocks for the 32 -> 32 layers).
        const int64_t stride = int64_t(CI) * kTaps * CO + CO;
        const int64_t want = std::min<int64_t>(std::min<int64_t>(kMaxPosBlocks, part_floats() / stride),
                                               ceil_div(nout, 64));
        const int per = int(ceil_div(nout, std::max<int64_t>(1, want)));
        const int nblk = int(ceil_div(nout, per));
        const dim3 wgrid(unsigned(nblk), unsigned(ceil_div(CI * kTaps, kBlock)));
        if (CO == kC && CI == kC)
            hipLaunchKernelGGL((k_conv_bwd_w_mfma<kC>), dim3(unsigned(nblk)), dim3(kBlock), 0, s, g, ns, dcur, lin,
                               per, n->part);
        else if (CO == kC && CI == 2)
            hipLaunchKernelGGL((k_conv_bwd_w_mfma<2>), dim3(unsigned(nblk)), dim3(kBlock), 0, s, g, ns, dcur, lin,
                               per, n->part);
        else if (CO == 1 && CI == kC)
            hipLaunchKernelGGL(k_conv_bwd_w1_mfma, dim3(unsigned(nblk)), dim3(kBlock), 0, s, g, ns, dcur, lin, per,
                               n->part);
        else
            hipLaunchKernelGGL((k_conv_bwd_w<1>), wgrid, dim3(kBlock), 0, s, g, ns, CI, dcur, lin, per, n->part);
        hipLaunchKernelGGL(k_fold_w, dim3(64), dim3(kBlock), 0, s, n->part, nblk, CI, CO, gw, gb);
        if (l > 0) {
            if (CO == kC) {
                // one column block per wave: two would keep too many gathers in registers
                hipLaunchKernelGGL((k_conv_bwd_data_mfma<1>), dim3(unsigned(ceil_div(nout, 128))), dim3(kBlock), 0, s,
                                   g, ns, dcur, W, n->act[l], dnext);
            } else {
                hipLaunchKernelGGL((k_conv_bwd_data<2>), dim3(unsigned(ceil_div(threads2, kBlock))), dim3(kBlock), 0,
                                   s, g, ns, CO, dcur, W, n->act[l], dnext);
            }
            std::swap(dcur, dnext);
        }
        FVX_HIP(hipGetLastError());
    }
    std::vector<float> lp(kLossBlocks);
    FVX_HIP(hipMemcpyAsync(lp.data(), n->lossp, 4 * kLossBlocks, hipMemcpyDeviceToHost, s));
    FVX_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (float v : lp) sum += double(v);
    return sum / double(nout);
}

struct Layout {
    size_t params, grads, m, v, act[5], g0, g1, part, lossp, scal, total;
};

Layout layout(int nx, int ny, int nz, int batch) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) / 256 * 256;
        return o;
    };
    const size_t cells = size_t(nx) * ny * nz, np = size_t(n_params()), B = size_t(batch);
    L.params = take(4 * np);
    L.grads = take(4 * np);
    L.m = take(4 * np);
    L.v = take(4 * np);
    L.act[0] = take(4 * B * 2 * cells);
    for (int l = 1; l <= 3; ++l) L.act[l] = take(4 * B * kC * cells);
    L.act[4] = take(4 * B * cells);
    L.g0 = take(4 * B * kC * cells);
    L.g1 = take(4 * B * kC * cells);
    L.part = take(4 * size_t(part_floats()));
    L.lossp = take(4 * kLossBlocks);
    L.scal = take(8 * 2);
    L.total = off;
    return L;
}

void check_dims(int nx, int ny, int nz, int batch) {
    FVX_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && batch >= 1, FVX_E_ARG, "net dimensions must be >= 1");
    FVX_REQUIRE(int64_t(nx) * ny * nz * batch * kC < (int64_t(1) << 31), FVX_E_ARG,
                "net too large for 32-bit activation indices (nx*ny*nz*batch*32 >= 2^31)");
}

void check_net(const fvx_net *n) { FVX_REQUIRE(n, FVX_E_ARG, "net is NULL"); }

void check_samples(const fvx_net *n, int ns) {
    FVX_REQUIRE(ns >= 1 && ns <= n->batch, FVX_E_ARG, "sample count must be in [1, batch]");
}

void check_op(const fvx_net *n, const fvx_op *op) {
    FVX_REQUIRE(op, FVX_E_ARG, "op is NULL");
    FVX_REQUIRE(op->grid_nx == n->nx && op->grid_ny == n->ny && op->k == n->nz, FVX_E_ARG,
                "operator is not the net's grid (Cartesian base nx x ny, k = nz)");
}

void zero(float *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(64), dim3(kBlock), 0, s, p, int(n));
    FVX_HIP(hipGetLastError());
}

void guess(fvx_net *n, const fvx_op *op, const double *B, const double *Pprev, double *X0, hipStream_t s) {
    const Grid g = grid_of(n);
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(1024), 0, s, g, B, op->ld, op->d64.area, 1.0 / op->dz,
                       int(op->singular), n->scal);
    hipLaunchKernelGGL(k_prepare, dim3(unsigned(std::min<int64_t>(1024, ceil_div(g.cells, kBlock)))), dim3(kBlock), 0,
                       s, g, B, Pprev, (const double *)nullptr, op->ld, op->d64.area, 1.0 / op->dz, n->scal,
                       n->act[0], (float *)nullptr);
    forward(n, 1, n->act[0], s);
    const unsigned out_blocks = unsigned(std::min<int64_t>(kGuessOutBlocks, ceil_div(int64_t(g.X) * g.Y, 1024)));
    hipLaunchKernelGGL(k_guess_out, dim3(out_blocks), dim3(1024), 0, s, g, n->act[4], n->scal, int(op->singular), X0,
                       op->ld);
    FVX_HIP(hipGetLastError());
}

}  // namespace net
}  // namespace fvx

using fvx::guard;
namespace N = fvx::net;

extern "C" {

int fvx_net_n_params(void) { return int(N::n_params()); }

int fvx_net_bytes(int nx, int ny, int nz, int batch, size_t *bytes) {
    return guard([&] {
        N::check_dims(nx, ny, nz, batch);
        FVX_REQUIRE(bytes, FVX_E_ARG, "bytes is NULL");
        *bytes = N::layout(nx, ny, nz, batch).total;
        return FVX_OK;
    });
}

int fvx_net_create(int nx, int ny, int nz, int batch, const float *init, void *dev_mem, size_t bytes, void *stream,
                   fvx_net **out) {
    return guard([&] {
        N::check_dims(nx, ny, nz, batch);
        FVX_REQUIRE(out && dev_mem, FVX_E_ARG, "NULL argument");
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(dev_mem) % 256 == 0, FVX_E_ARG, "dev_mem must be 256-byte aligned");
        const N::Layout L = N::layout(nx, ny, nz, batch);
        FVX_REQUIRE(bytes >= L.total, FVX_E_NOMEM, "net buffer too small: need " + std::to_string(L.total));
        auto n = std::make_unique<fvx_net>();
        char *b = static_cast<char *>(dev_mem);
        n->nx = nx;
        n->ny = ny;
        n->nz = nz;
        n->batch = batch;
        n->cells = nx * ny * nz;
        auto f = [&](size_t off) { return reinterpret_cast<float *>(b + off); };
        n->params = f(L.params);
        n->grads = f(L.grads);
        n->m = f(L.m);
        n->v = f(L.v);
        for (int l = 0; l < 5; ++l) n->act[l] = f(L.act[l]);
        n->g0 = f(L.g0);
        n->g1 = f(L.g1);
        n->part = f(L.part);
        n->lossp = f(L.lossp);
        n->scal = reinterpret_cast<double *>(b + L.scal);
        hipStream_t s = fvx::as_stream(stream);
        const int64_t np = N::n_params();
        if (init)
            FVX_HIP(hipMemcpyAsync(n->params, init, 4 * size_t(np), hipMemcpyHostToDevice, s));
        else
            N::zero(n->params, np, s);
        N::zero(n->grads, np, s);
        N::zero(n->m, np, s);
        N::zero(n->v, np, s);
        FVX_HIP(hipStreamSynchronize(s));
        *out = n.release();
        return FVX_OK;
    });
}

int fvx_net_destroy(fvx_net *n) {
    delete n;
    return FVX_OK;
}

int fvx_net_get_params(const fvx_net *n, float *params, float *grads) {
    return guard([&] {
        N::check_net(n);
        const size_t np = size_t(N::n_params());
        if (params) FVX_HIP(hipMemcpy(params, n->params, 4 * np, hipMemcpyDeviceToHost));
        if (grads) FVX_HIP(hipMemcpy(grads, n->grads, 4 * np, hipMemcpyDeviceToHost));
        return FVX_OK;
    });
}

int fvx_net_set_params(fvx_net *n, const float *params, void *stream) {
    return guard([&] {
        N::check_net(n);
        FVX_REQUIRE(params, FVX_E_ARG, "params is NULL");
        hipStream_t s = fvx::as_stream(stream);
        const int64_t np = N::n_params();
        FVX_HIP(hipMemcpyAsync(n->params, params, 4 * size_t(np), hipMemcpyHostToDevice, s));
        N::zero(n->m, np, s);
        N::zero(n->v, np, s);
        FVX_HIP(hipStreamSynchronize(s));
        n->step = 0;
        return FVX_OK;
    });
}

namespace {
constexpr char kNetMagic[8] = {'F', 'V', 'X', 'N', 'E', 'T', '0', '1'};

struct FileCloser {
    void operator()(FILE *f) const {
        if (f) std::fclose(f);
    }
};
}  // namespace

int fvx_net_save(const fvx_net *n, const char *path, void *stream) {
    return guard([&] {
        N::check_net(n);
        FVX_REQUIRE(path, FVX_E_ARG, "path is NULL");
        const size_t np = size_t(N::n_params());
        FVX_HIP(hipStreamSynchronize(fvx::as_stream(stream)));
        std::vector<float> host(3 * np);
        FVX_HIP(hipMemcpy(host.data(), n->params, 4 * np, hipMemcpyDeviceToHost));
        FVX_HIP(hipMemcpy(host.data() + np, n->m, 4 * np, hipMemcpyDeviceToHost));
        FVX_HIP(hipMemcpy(host.data() + 2 * np, n->v, 4 * np, hipMemcpyDeviceToHost));
        std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "wb"));
        FVX_REQUIRE(f, FVX_E_IO, std::string("cannot open ") + path + " for writing");
        const int32_t head[2] = {int32_t(np), int32_t(n->step)};
        bool ok = std::fwrite(kNetMagic, 1, 8, f.get()) == 8 && std::fwrite(head, 4, 2, f.get()) == 2 &&
                  std::fwrite(host.data(), 4, host.size(), f.get()) == host.size();
        ok = std::fclose(f.release()) == 0 && ok;
        FVX_REQUIRE(ok, FVX_E_IO, std::string("writing ") + path + " failed");
        return FVX_OK;
    });
}

int fvx_net_load(fvx_net *n, const char *path, void *stream) {
    return guard([&] {
        N::check_net(n);
        FVX_REQUIRE(path, FVX_E_ARG, "path is NULL");
        const size_t np = size_t(N::n_params());
        std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "rb"));
        FVX_REQUIRE(f, FVX_E_IO, std::string("cannot open ") + path);
        char magic[8];
        int32_t head[2];
        FVX_REQUIRE(std::fread(magic, 1, 8, f.get()) == 8 && std::memcmp(magic, kNetMagic, 8) == 0, FVX_E_IO,
                    std::string(path) + " is not a network checkpoint");
        FVX_REQUIRE(std::fread(head, 4, 2, f.get()) == 2 && head[0] == int32_t(np) && head[1] >= 0, FVX_E_IO,
                    std::string(path) + ": parameter count " + std::to_string(head[0]) + ", this network has " +
                        std::to_string(np));
        std::vector<float> host(3 * np);
        FVX_REQUIRE(std::fread(host.data(), 4, host.size(), f.get()) == host.size(), FVX_E_IO,
                    std::string(path) + " is truncated");
        hipStream_t s = fvx::as_stream(stream);
        FVX_HIP(hipMemcpyAsync(n->params, host.data(), 4 * np, hipMemcpyHostToDevice, s));
        FVX_HIP(hipMemcpyAsync(n->m, host.data() + np, 4 * np, hipMemcpyHostToDevice, s));
        FVX_HIP(hipMemcpyAsync(n->v, host.data() + 2 * np, 4 * np, hipMemcpyHostToDevice, s));
        FVX_HIP(hipStreamSynchronize(s));
        n->step = head[1];
        return FVX_OK;
    });
}

int fvx_net_forward(fvx_net *n, int ns, const float *in, float *out, void *stream) {
    return guard([&] {
        N::check_net(n);
        N::check_samples(n, ns);
        FVX_REQUIRE(in && out, FVX_E_ARG, "NULL input or output");
        hipStream_t s = fvx::as_stream(stream);
        N::forward(n, ns, in, s);
        FVX_HIP(hipMemcpyAsync(out, n->act[4], 4 * size_t(ns) * n->cells, hipMemcpyDeviceToDevice, s));
        return FVX_OK;
    });
}

int fvx_net_gradients(fvx_net *n, int ns, const float *in, const float *target, double *loss, void *stream) {
    return guard([&] {
        N::check_net(n);
        N::check_samples(n, ns);
        FVX_REQUIRE(in && target, FVX_E_ARG, "NULL input or target");
        const double l = N::backward(n, ns, in, target, fvx::as_stream(stream));
        if (loss) *loss = l;
        return FVX_OK;
    });
}

static void apply_adam(fvx_net *n, float lr, hipStream_t s) {
    n->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = float(1.0 - std::pow(b1, n->step)), c2 = float(1.0 - std::pow(b2, n->step));
    hipLaunchKernelGGL(N::k_adam, dim3(64), dim3(N::kBlock), 0, s, n->params, n->grads, n->m, n->v,
                       int(N::n_params()), lr, float(b1), float(b2), 1e-8f, c1, c2);
    FVX_HIP(hipGetLastError());
}

int fvx_net_train_step(fvx_net *n, int ns, const float *in, const float *target, float lr, double *loss,
                       void *stream) {
    return guard([&] {
        N::check_net(n);
        N::check_samples(n, ns);
        FVX_REQUIRE(in && target, FVX_E_ARG, "NULL input or target");
        FVX_REQUIRE(lr > 0.0f && std::isfinite(lr), FVX_E_ARG, "lr must be positive");
        hipStream_t s = fvx::as_stream(stream);
        const double l = N::backward(n, ns, in, target, s);
        apply_adam(n, lr, s);
        if (loss) *loss = l;
        return FVX_OK;
    });
}

float *fvx_net_grads(fvx_net *n) { return n ? n->grads : nullptr; }

int fvx_net_apply_adam(fvx_net *n, float lr, void *stream) {
    return guard([&] {
        N::check_net(n);
        FVX_REQUIRE(lr > 0.0f && std::isfinite(lr), FVX_E_ARG, "lr must be positive");
        apply_adam(n, lr, fvx::as_stream(stream));
        return FVX_OK;
    });
}

int fvx_net_prepare(fvx_net *n, const fvx_op *op, const double *B, const double *Pprev, const double *Xstar,
                    float *in, float *target, void *stream) {
    return guard([&] {
        N::check_net(n);
        N::check_op(n, op);
        FVX_REQUIRE(B && in && (target == nullptr) == (Xstar == nullptr), FVX_E_ARG,
                    "NULL B or input, or only one of target and Xstar");
        hipStream_t s = fvx::as_stream(stream);
        const N::Grid g = N::grid_of(n);
        hipLaunchKernelGGL(N::k_scale, dim3(1), dim3(1024), 0, s, g, B, op->ld, op->d64.area, 1.0 / op->dz,
                           int(op->singular), n->scal);
        hipLaunchKernelGGL(N::k_prepare, dim3(unsigned(std::min<int64_t>(1024, fvx::ceil_div(g.cells, N::kBlock)))),
                           dim3(N::kBlock), 0, s, g, B, Pprev, Xstar, op->ld, op->d64.area, 1.0 / op->dz, n->scal,
                           in, target);
        FVX_HIP(hipGetLastError());
        return FVX_OK;
    });
}

int fvx_net_guess(fvx_net *n, const fvx_op *op, const double *B, const double *Pprev, double *X0, void *stream) {
    return guard([&] {
        N::check_net(n);
        N::check_op(n, op);
        FVX_REQUIRE(B && X0, FVX_E_ARG, "NULL argument");
        N::guess(n, op, B, Pprev, X0, fvx::as_stream(stream));
        return FVX_OK;
    });
}

int fvx_poisson_solve_net(const fvx_op *op, fvx_net *n, const double *B, const double *Pprev, double *X,
                          const fvx_solve_opts *opts, void *ws, size_t ws_bytes, fvx_solve_stats *stats,
                          int *source, void *stream) {
    const auto t0 = std::chrono::steady_clock::now();
    fvx_solve_opts o{};
    const int rc = guard([&]() -> int {
        N::check_net(n);
        N::check_op(n, op);
        FVX_REQUIRE(B && X && opts && ws, FVX_E_ARG, "NULL argument");
        size_t need = 0;
        const int q = fvx_solve_bytes(op, opts, &need);
        if (q != FVX_OK) return q;
        FVX_REQUIRE(ws_bytes >= need, FVX_E_NOMEM, "workspace too small: need " + std::to_string(need));
        FVX_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, FVX_E_ARG, "ws must be 256-byte aligned");
        hipStream_t s = fvx::as_stream(stream);
        N::guess(n, op, B, Pprev, X, s);
        // Candidates judged by their residual: the network's guess, the
        // previous pressure, and zero (ratio 1).
        double best = fvx::guess_residual_ratio(op, B, X, ws, s);
        int src = FVX_GUESS_NET;
        if (!(best < 1.0)) {
            best = 1.0;
            src = FVX_GUESS_ZERO;
        }
        if (Pprev) {
            const double rp = fvx::guess_residual_ratio(op, B, Pprev, ws, s);
            if (rp < best) {
                best = rp;
                src = FVX_GUESS_GIVEN;
                FVX_HIP(hipMemcpyAsync(X, Pprev, sizeof(double) * size_t(op->n_b) * op->ld, hipMemcpyDeviceToDevice,
                                       s));
            }
        }
        o = *opts;
        o.guess = src == FVX_GUESS_ZERO ? FVX_GUESS_ZERO : FVX_GUESS_GIVEN;
        if (source) *source = src;
        return FVX_OK;
    });
    if (rc != FVX_OK) return rc;
    const int st = fvx_poisson_solve(op, B, X, &o, ws, ws_bytes, stats, stream);
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

}  // extern "C"
