// Learned preconditioner: a 4-layer convolutional network with 3^4 kernels acting on the odd-site
// half field of the even-odd system, one s-slice at a time with weights shared over s.
//
// Activations are rows of 32 channels (complex-as-real spin x colour = 24, padded to 32 for the
// matrix cores), row = cb * Ns + s.  The 4D geometry is the checkerboard-compressed lattice
// (xh, y, z, t) with periodic wrap.  Every layer is an implicit GEMM
//     Y[row][n] = b[n] + sum_{tap < 81} sum_{k < 32} X[nbr(row, tap)][k] W[tap][n][k]
// on v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation).  The weight gradient is a GEMM
// whose reduction runs over rows; it uses channel-major copies of X and dY so that 8 consecutive
// rows of one channel are one 16-byte operand.
#include "eofa_int.h"
#include "cnn.h"

namespace eofa {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float f) {
    // round to nearest even
    unsigned u = __builtin_bit_cast(unsigned, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }

// cb-compressed coordinates of a 4D checkerboard index
struct CbGeom {
    int Lxh, Ly, Lz, Lt, Ns;
    int Vh;
};

// per-lane offsets of the three neighbours per dimension: off[d][0..2] for shifts -1, 0, +1
__device__ __forceinline__ void cb_offsets(const CbGeom& g, int cb, int off[4][3]) {
    int xh = cb % g.Lxh, r = cb / g.Lxh;
    int y = r % g.Ly; r /= g.Ly;
    int z = r % g.Lz;
    int t = r / g.Lz;
    const int sy = g.Lxh, sz = g.Lxh * g.Ly, st = sz * g.Lz;
#pragma unroll
    for (int d = -1; d <= 1; d++) {
        off[0][d + 1] = (xh + d + g.Lxh) % g.Lxh;
        off[1][d + 1] = ((y + d + g.Ly) % g.Ly) * sy;
        off[2][d + 1] = ((z + d + g.Lz) % g.Lz) * sz;
        off[3][d + 1] = ((t + d + g.Lt) % g.Lt) * st;
    }
}

// tap = 27 (dt+1) + 9 (dz+1) + 3 (dy+1) + (dx+1); its mirror (-d) is 80 - tap.
__device__ __forceinline__ int tap_cb(const int off[4][3], int tap) {
    return off[0][tap % 3] + off[1][(tap / 3) % 3] + off[2][(tap / 9) % 3] + off[3][tap / 27];
}

// -------------------------------------------------------------------- forward conv
// One wave computes 64 rows x 32 output channels (4 row tiles x 2 column tiles of 16x16).
// X: [rows][32] bf16; W: [81][32 n][32 k] bf16; bias [32] f32 (may be null); Y: [rows][32] bf16 or f32.
template <bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv_fwd(const unsigned short* __restrict__ X,
                                                  const unsigned short* __restrict__ W,
                                                  const float* __restrict__ bias, void* __restrict__ Y, CbGeom g,
                                                  int rows, int relu) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 4) + (threadIdx.x >> 6);
    const int row0 = wave * 64;
    if (row0 >= rows) return;
    const int li = lane & 15;   // row within a tile (A) / column within a tile (B, D)
    const int kb = lane >> 4;   // which 8-wide k block
    int off[4][4][3];
    int srow[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        int r = row0 + t * 16 + li;
        if (r >= rows) r = rows - 1;
        const int cb = r / g.Ns;
        srow[t] = r - cb * g.Ns;
        cb_offsets(g, cb, off[t]);
    }
    f32x4 acc[4][2];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        acc[t][0] = {0, 0, 0, 0};
        acc[t][1] = {0, 0, 0, 0};
    }
    for (int tap = 0; tap < 81; tap++) {
        const unsigned short* wt = W + (size_t)tap * 1024;
        const bf16x8 b0 = *(const bf16x8*)(wt + li * 32 + kb * 8);
        const bf16x8 b1 = *(const bf16x8*)(wt + (16 + li) * 32 + kb * 8);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int nrow = tap_cb(off[t], tap) * g.Ns + srow[t];
            const bf16x8 a = *(const bf16x8*)(X + (size_t)nrow * 32 + kb * 8);
            acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[t][0], 0, 0, 0);
            acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[t][1], 0, 0, 0);
        }
    }
    // D layout: lane holds rows 4*kb + j (j < 4) of the tile, column li (+16 for the second half)
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int n = h * 16 + li;
            const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int r = row0 + t * 16 + kb * 4 + j;
                if (r >= rows) continue;
                float v = acc[t][h][j] + bn;
                if (relu && v < 0.0f) v = 0.0f;
                if constexpr (OUT_F32) ((float*)Y)[(size_t)r * 32 + n] = v;
                else ((unsigned short*)Y)[(size_t)r * 32 + n] = bf16_bits(v);
            }
        }
}

// -------------------------------------------------------------------- forward conv, LDS-tiled
// A workgroup (2 waves) owns a 4 x 4 x 2 x 2 block of compressed sites (xh, y, z, t) and 2 s-slices
// = 128 rows.  It stages the block with its one-site halo (6 x 6 x 4 x 4 sites x 2 slices x 64 B =
// 72 KB) in LDS once, then every tap reads its A operands from LDS: global traffic is the halo
// (9x the block) instead of one gathered row block per tap (81x).  Needs Lxh % 4 == 0, Ly % 4 == 0,
// Lz, Lt, Ns even.
constexpr int CT_X = 4, CT_Y = 4, CT_Z = 2, CT_T = 2, CT_S = 2;
constexpr int CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2, CH_T = CT_T + 2;
constexpr int CH_SITES = CH_X * CH_Y * CH_Z * CH_T;  // 576
constexpr int CT_ROWS = CT_X * CT_Y * CT_Z * CT_T * CT_S;  // 128

template <bool OUT_F32>
__global__ __launch_bounds__(128) void k_conv_fwd_lds(const unsigned short* __restrict__ X,
                                                      const unsigned short* __restrict__ W,
                                                      const float* __restrict__ bias, void* __restrict__ Y, CbGeom g,
                                                      int relu) {
    // 16-byte units: [halo site][slice][4 k-blocks]
    __shared__ uint4 lds[CH_SITES * CT_S * 4];
    const int nbx = g.Lxh / CT_X, nby = g.Ly / CT_Y, nbz = g.Lz / CT_Z, nbt = g.Lt / CT_T;
    int b = blockIdx.x;
    const int bx = b % nbx; b /= nbx;
    const int by = b % nby; b /= nby;
    const int bz = b % nbz; b /= nbz;
    const int bt = b % nbt; b /= nbt;
    const int s0 = b * CT_S;
    const int x0 = bx * CT_X, y0 = by * CT_Y, z0 = bz * CT_Z, t0 = bt * CT_T;
    // stage: halo site h -> its 2 rows (128 contiguous bytes) = 8 chunks of 16 B; 36 chunks per thread,
    // loaded in batches of 12 independent loads (wrap by compare, no integer division by the extents)
    auto wrap = [](int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); };
    constexpr int PER = CH_SITES * 8 / 128, BATCH = 12;
    static_assert(PER % BATCH == 0, "staging batches");
#pragma unroll
    for (int i0 = 0; i0 < PER; i0 += BATCH) {
        uint4 v[BATCH];
#pragma unroll
        for (int i = 0; i < BATCH; i++) {
            const int c = threadIdx.x + 128 * (i0 + i);
            int h = c >> 3;
            const int part = c & 7;
            const int hx = h % CH_X; h /= CH_X;
            const int hy = h % CH_Y; h /= CH_Y;
            const int hz = h % CH_Z;
            const int ht = h / CH_Z;
            const int gx = wrap(x0 + hx - 1, g.Lxh), gy = wrap(y0 + hy - 1, g.Ly);
            const int gz = wrap(z0 + hz - 1, g.Lz), gt = wrap(t0 + ht - 1, g.Lt);
            const size_t cb = (size_t)gx + (size_t)g.Lxh * (gy + (size_t)g.Ly * (gz + (size_t)g.Lz * gt));
            v[i] = *(const uint4*)(X + (cb * g.Ns + s0) * 32 + part * 8);
        }
#pragma unroll
        for (int i = 0; i < BATCH; i++) lds[threadIdx.x + 128 * (i0 + i)] = v[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15, kb = lane >> 4;
    // tile rows: r = site * 2 + slice, site = ((lt * CT_Z + lz) * CT_Y + ly) * CT_X + lx; wave w owns rows [64w, 64w+64)
    int abase[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int r = wave * 64 + t * 16 + li;
        const int sl = r & 1;
        int site = r >> 1;
        const int lx = site % CT_X; site /= CT_X;
        const int ly = site % CT_Y; site /= CT_Y;
        const int lz = site % CT_Z;
        const int lt = site / CT_Z;
        const int hs = (lx + 1) + CH_X * ((ly + 1) + CH_Y * ((lz + 1) + CH_Z * (lt + 1)));
        abase[t] = (hs * CT_S + sl) * 4 + kb;
    }
    f32x4 acc[4][2];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        acc[t][0] = {0, 0, 0, 0};
        acc[t][1] = {0, 0, 0, 0};
    }
    // the weights of the next (dt, dz, dy) group of 3 taps are in flight while this group computes
    const unsigned short* wl = W + li * 32 + kb * 8;
    bf16x8 bw[3][2];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        bw[d][0] = *(const bf16x8*)(wl + (size_t)d * 1024);
        bw[d][1] = *(const bf16x8*)(wl + (size_t)d * 1024 + 512);
    }
    // A fragments of a (dt, dz, dy) group of 3 taps: [dx][row tile]; the next group's are read from LDS
    // while this group's 24 MFMAs run
    auto load_group = [&](int tq, uint4 (*a)[4]) {
        const int dy = tq % 3 - 1, dz = (tq / 3) % 3 - 1, dt = tq / 9 - 1;
        const int off_yzt = CH_X * (dy + CH_Y * (dz + CH_Z * dt));
#pragma unroll
        for (int dx = -1; dx <= 1; dx++)
#pragma unroll
            for (int t = 0; t < 4; t++) a[dx + 1][t] = lds[abase[t] + (off_yzt + dx) * CT_S * 4];
    };
    uint4 acur[3][4], anext[3][4];
    load_group(0, acur);
    for (int tq = 0; tq < 27; tq++) {
        bf16x8 bn[3][2];
        const int tn = (tq < 26 ? tq + 1 : tq);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            bn[d][0] = *(const bf16x8*)(wl + (size_t)(3 * tn + d) * 1024);
            bn[d][1] = *(const bf16x8*)(wl + (size_t)(3 * tn + d) * 1024 + 512);
        }
        load_group(tn, anext);
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const bf16x8 a = __builtin_bit_cast(bf16x8, acur[d][t]);
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[d][0], acc[t][0], 0, 0, 0);
                acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[d][1], acc[t][1], 0, 0, 0);
            }
#pragma unroll
        for (int d = 0; d < 3; d++) {
            bw[d][0] = bn[d][0];
            bw[d][1] = bn[d][1];
#pragma unroll
            for (int t = 0; t < 4; t++) acur[d][t] = anext[d][t];
        }
    }
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int n = h * 16 + li;
            const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int r = wave * 64 + t * 16 + kb * 4 + j;
                const int sl = r & 1;
                int site = r >> 1;
                const int lx = site % CT_X; site /= CT_X;
                const int ly = site % CT_Y; site /= CT_Y;
                const int lz = site % CT_Z;
                const int lt = site / CT_Z;
                const size_t cb = (size_t)(x0 + lx) +
                                  (size_t)g.Lxh * ((y0 + ly) + (size_t)g.Ly * ((z0 + lz) + (size_t)g.Lz * (t0 + lt)));
                const size_t row = cb * g.Ns + s0 + sl;
                float v = acc[t][h][j] + bn;
                if (relu && v < 0.0f) v = 0.0f;
                if constexpr (OUT_F32) ((float*)Y)[row * 32 + n] = v;
                else ((unsigned short*)Y)[row * 32 + n] = bf16_bits(v);
            }
        }
}

static bool conv_tiles(const CbGeom& g) {
    return g.Lxh % CT_X == 0 && g.Ly % CT_Y == 0 && g.Lz % CT_Z == 0 && g.Lt % CT_T == 0 && g.Ns % CT_S == 0;
}

// -------------------------------------------------------------------- weight gradient
// dW[tap][n][k] = sum_rows dY[row][n] X[nbr(row, tap)][k], from channel-major dYT [32][rows] and
// XT [32][rows] (bf16), so that 8 consecutive rows of one channel (one site, 8 consecutive s when
// Ns % 8 == 0) are one 16-byte operand.  Partials go to part[chunk][tap][32][32].
// Block (chunk, tq) computes the three taps (dt, dz, dy) = tq,
// dx = -1, 0, 1, each wave the full 32 x 32 of all three over a quarter of the chunk's rows (one dY
// operand pair feeds 12 MFMAs), then the four waves' sums are added in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_conv_wgrad3(const unsigned short* __restrict__ dYT,
                                                     const unsigned short* __restrict__ XT, float* __restrict__ part,
                                                     CbGeom g, int rows, int chunk_rows) {
    const int tq = blockIdx.y;
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, kb = lane >> 4;
    const int dy = tq % 3 - 1, dz = (tq / 3) % 3 - 1, dt = tq / 9 - 1;
    f32x4 acc[3][2][2];  // [dx][n tile][k tile]
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            acc[a][b][0] = {0, 0, 0, 0};
            acc[a][b][1] = {0, 0, 0, 0};
        }
    const int quarter = chunk_rows / 4;  // multiple of 32
    const int r_begin = chunk * chunk_rows + w * quarter;
    const int r_end = min(rows, r_begin + quarter);
    const int sy = g.Lxh, sz = g.Lxh * g.Ly, st = sz * g.Lz;
    // operands of the 32 rows at rb (zeros past r_end); the next step's are requested before this step's
    // 12 MFMAs, so a global round trip overlaps the matrix-core work
    auto load_ops = [&](int rb, bf16x8& a0, bf16x8& a1, bf16x8 (*b)[2]) {
        const int r8 = rb + kb * 8;  // 8 rows (one site, 8 consecutive s) of this lane's k block
        if (r8 + 8 <= r_end) {
            a0 = *(const bf16x8*)(dYT + (size_t)li * rows + r8);
            a1 = *(const bf16x8*)(dYT + (size_t)(16 + li) * rows + r8);
            const int cb = r8 / g.Ns, sl = r8 - cb * g.Ns;
            int xh = cb % g.Lxh, q = cb / g.Lxh;
            const int y = q % g.Ly; q /= g.Ly;
            const int z = q % g.Lz;
            const int t = q / g.Lz;
            const int yzt = ((y + dy + g.Ly) % g.Ly) * sy + ((z + dz + g.Lz) % g.Lz) * sz + ((t + dt + g.Lt) % g.Lt) * st;
#pragma unroll
            for (int dx = -1; dx <= 1; dx++) {
                const int nrow = (yzt + (xh + dx + g.Lxh) % g.Lxh) * g.Ns + sl;
                b[dx + 1][0] = *(const bf16x8*)(XT + (size_t)li * rows + nrow);
                b[dx + 1][1] = *(const bf16x8*)(XT + (size_t)(16 + li) * rows + nrow);
            }
        } else {
            for (int j = 0; j < 8; j++) {
                a0[j] = (__bf16)0.0f; a1[j] = (__bf16)0.0f;
                for (int d = 0; d < 3; d++) { b[d][0][j] = (__bf16)0.0f; b[d][1][j] = (__bf16)0.0f; }
            }
        }
    };
    bf16x8 a0, a1, b[3][2];
    load_ops(r_begin, a0, a1, b);
    for (int rb = r_begin; rb < r_end; rb += 32) {
        bf16x8 a0n, a1n, bn[3][2];
        load_ops(rb + 32, a0n, a1n, bn);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            acc[d][0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[d][0], acc[d][0][0], 0, 0, 0);
            acc[d][0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[d][1], acc[d][0][1], 0, 0, 0);
            acc[d][1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[d][0], acc[d][1][0], 0, 0, 0);
            acc[d][1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[d][1], acc[d][1][1], 0, 0, 0);
        }
        a0 = a0n;
        a1 = a1n;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            b[d][0] = bn[d][0];
            b[d][1] = bn[d][1];
        }
    }
    // waves 1..3 park their sums in LDS, wave 0 adds them in order and writes the partial
    __shared__ float red[3][3 * 1024];
    if (w > 0) {
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int nt = 0; nt < 2; nt++)
#pragma unroll
                for (int kt = 0; kt < 2; kt++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        red[w - 1][d * 1024 + (nt * 16 + kb * 4 + j) * 32 + kt * 16 + li] = acc[d][nt][kt][j];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            float* dst = part + ((size_t)chunk * 81 + tq * 3 + d) * 1024;
#pragma unroll
            for (int nt = 0; nt < 2; nt++)
#pragma unroll
                for (int kt = 0; kt < 2; kt++)
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int e = (nt * 16 + kb * 4 + j) * 32 + kt * 16 + li;
                        dst[e] = ((acc[d][nt][kt][j] + red[0][d * 1024 + e]) + red[1][d * 1024 + e]) + red[2][d * 1024 + e];
                    }
        }
    }
}

// sum over chunks (fixed order) -> g[tap][n][k], masked to the live channels
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nchunk, float* __restrict__ gw,
                                                      int cin, int cout) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 81 * 1024) return;
    const int n = (i / 32) % 32, k = i % 32;
    float s = 0.0f;
    for (int c = 0; c < nchunk; c++) s += part[(size_t)c * 81 * 1024 + i];
    gw[i] = (n < cout && k < cin) ? s : 0.0f;
}

// bias gradient gb[n] = sum_rows dY[row][n], in two fixed-order stages: block b sums rows
// b*8 + (tid/32) + k*8*gridDim into part[b][n] (coalesced: 8 rows x 32 channels per step), then one
// block adds the partials.
constexpr int BGRAD_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_bgrad_part(const float* __restrict__ dY, int rows, double* __restrict__ part) {
    const int n = threadIdx.x & 31, r0 = threadIdx.x >> 5;
    double s = 0.0;
    for (size_t r = (size_t)blockIdx.x * 8 + r0; r < (size_t)rows; r += (size_t)8 * gridDim.x) s += dY[r * 32 + n];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 32) {
        double t = 0.0;
        for (int k = 0; k < 8; k++) t += red[k * 32 + n];
        part[(size_t)blockIdx.x * 32 + n] = t;
    }
}
__global__ __launch_bounds__(32) void k_bgrad_fin(const double* __restrict__ part, int nb, float* __restrict__ gb, int cout) {
    const int n = threadIdx.x;
    double t = 0.0;
    for (int b = 0; b < nb; b++) t += part[(size_t)b * 32 + n];
    gb[n] = (n < cout) ? (float)t : 0.0f;
}

// -------------------------------------------------------------------- elementwise helpers
// [rows][32] (bf16 or f32) -> channel-major [32][rows] bf16, through a 64-row LDS tile (reads and writes
// both coalesced)
template <bool IN_F32>
__global__ __launch_bounds__(256) void k_to_chmajor(const void* __restrict__ in, unsigned short* __restrict__ out, int rows) {
    __shared__ unsigned short tile[32][64 + 2];
    const size_t r0 = (size_t)blockIdx.x * 64;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int e = threadIdx.x + 256 * k;  // 2048 elements: row e / 32, channel e % 32
        const int rr = e >> 5, c = e & 31;
        const size_t r = r0 + rr;
        float v = 0.0f;
        if (r < (size_t)rows)
            v = IN_F32 ? ((const float*)in)[r * 32 + c] : bf16_float(((const unsigned short*)in)[r * 32 + c]);
        tile[c][rr] = bf16_bits(v);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int e = threadIdx.x + 256 * k;  // channel e / 64, row e % 64
        const int c = e >> 6, rr = e & 63;
        const size_t r = r0 + rr;
        if (r < (size_t)rows) out[(size_t)c * rows + r] = tile[c][rr];
    }
}

// f32 -> bf16 (same layout)
__global__ __launch_bounds__(256) void k_f32_to_bf16(const float* __restrict__ in, unsigned short* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) out[i] = bf16_bits(in[i]);
}

// ReLU backward: dX *= (Xpre > 0)  (Xpre = the layer output before ReLU, kept in bf16)
__global__ __launch_bounds__(256) void k_relu_bwd(float* __restrict__ d, const unsigned short* __restrict__ act, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        if (bf16_float(act[i]) <= 0.0f) d[i] = 0.0f;
}

// Weights for the backward-data convolution: Wt[tap][k][n] = W[80 - tap][n][k]
__global__ __launch_bounds__(256) void k_w_transpose(const float* __restrict__ w, unsigned short* __restrict__ wt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 81 * 1024) return;
    const int tap = i / 1024, k = (i / 32) % 32, n = i % 32;
    wt[i] = bf16_bits(w[(size_t)(80 - tap) * 1024 + n * 32 + k]);
}

// Adam on the FP32 master parameters
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ gsum, float* __restrict__ m,
                                              float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2, float gscale) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float gi = gsum[i] * gscale;
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// half field [cb][12][Ns] (complex double) -> rows [cb*Ns + s][32] bf16 scaled by sc (24 live channels)
__global__ __launch_bounds__(256) void k_half_to_rows(const cd* __restrict__ h, unsigned short* __restrict__ X, int Vh,
                                                      int Ns, const double* __restrict__ scale_ptr, int inv) {
    const double sc = inv ? 1.0 / sqrt(*scale_ptr) : *scale_ptr;
    const size_t n = (size_t)Vh * Ns * 32;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int c = (int)(i % 32);
        const size_t row = i / 32;
        const int s = (int)(row % Ns);
        const size_t cb = row / Ns;
        float v = 0.0f;
        if (c < 24) {
            const cd z = h[(cb * 12 + (c >> 1)) * Ns + s];
            v = (float)(sc * ((c & 1) ? z.y : z.x));
        }
        X[i] = bf16_bits(v);
    }
}

// rows [row][32] f32 -> half field (complex double) times sqrt(*scale) (the norm of the network input)
__global__ __launch_bounds__(256) void k_rows_to_half(const float* __restrict__ Y, cd* __restrict__ h, int Vh, int Ns,
                                                      const double* __restrict__ scale_ptr) {
    const double sc = sqrt(*scale_ptr);
    const size_t n = (size_t)Vh * 12 * Ns;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int s = (int)(i % Ns);
        const int j = (int)((i / Ns) % 12);
        const size_t cb = i / ((size_t)12 * Ns);
        const size_t row = cb * Ns + s;
        h[i] = {sc * Y[row * 32 + 2 * j], sc * Y[row * 32 + 2 * j + 1]};
    }
}

// dY = (Y - T) * w for the MSE loss; also the partial sums of |Y - T|^2 (T: target rows in f32)
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                                             size_t n, float w, Red red) {
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float d = Y[i] - T[i];
        dY[i] = d * w;
        s += (double)d * d;
    }
    __shared__ double lds[4];
    finish_sum(red, block_sum256(s, lds));
}

// half field -> f32 rows scaled by 1/sqrt(*scale_ptr) (targets)
__global__ __launch_bounds__(256) void k_half_to_rows_f32(const cd* __restrict__ h, float* __restrict__ T, int Vh, int Ns,
                                                          const double* __restrict__ scale_ptr) {
    const double sc = 1.0 / sqrt(*scale_ptr);
    const size_t n = (size_t)Vh * Ns * 32;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int c = (int)(i % 32);
        const size_t row = i / 32;
        const int s = (int)(row % Ns);
        const size_t cb = row / Ns;
        float v = 0.0f;
        if (c < 24) {
            const cd z = h[(cb * 12 + (c >> 1)) * Ns + s];
            v = (float)(sc * ((c & 1) ? z.y : z.x));
        }
        T[i] = v;
    }
}

// ==================================================================== launchers
static inline int grid_for(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b ? b : 1));
}

static CbGeom cbg(const Geom& g, int Ns) { return CbGeom{g.Lxh, g.Ly, g.Lz, g.Lt, Ns, g.Vh}; }


hipError_t cnn_conv_fwd(const unsigned short* X, const unsigned short* W, const float* bias, void* Y, bool out_f32,
                        const Geom& g, int Ns, int relu, hipStream_t st) {
    const CbGeom cg = cbg(g, Ns);
    if (conv_tiles(cg)) {
        const int nblk = g.Vh * Ns / CT_ROWS;
        if (out_f32) hipLaunchKernelGGL(k_conv_fwd_lds<true>, dim3(nblk), dim3(128), 0, st, X, W, bias, Y, cg, relu);
        else hipLaunchKernelGGL(k_conv_fwd_lds<false>, dim3(nblk), dim3(128), 0, st, X, W, bias, Y, cg, relu);
        return hipGetLastError();
    }
    const int rows = g.Vh * Ns;
    const int waves = (rows + 63) / 64;
    const int grid = (waves + 3) / 4;
    if (out_f32) hipLaunchKernelGGL(k_conv_fwd<true>, dim3(grid), dim3(256), 0, st, X, W, bias, Y, cbg(g, Ns), rows, relu);
    else hipLaunchKernelGGL(k_conv_fwd<false>, dim3(grid), dim3(256), 0, st, X, W, bias, Y, cbg(g, Ns), rows, relu);
    return hipGetLastError();
}

hipError_t cnn_wgrad(const unsigned short* dYT, const unsigned short* XT, float* part, float* gw, const Geom& g, int Ns,
                     int cin, int cout, hipStream_t st) {
    const int rows = g.Vh * Ns;
    const int nchunk = cnn_wgrad_chunks(rows);
    const int chunk_rows = (rows + nchunk - 1) / nchunk;
    // each of the 4 waves takes a quarter of the chunk: chunk rows a multiple of 128
    hipLaunchKernelGGL(k_conv_wgrad3, dim3(nchunk, 27), dim3(256), 0, st, dYT, XT, part, cbg(g, Ns), rows,
                       (chunk_rows + 127) / 128 * 128);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((81 * 1024 + 255) / 256), dim3(256), 0, st, part, nchunk, gw, cin, cout);
    return hipGetLastError();
}

int cnn_wgrad_chunks(int rows) {
    int c = rows / 4096;
    return c < 1 ? 1 : (c > 256 ? 256 : c);
}

hipError_t cnn_bgrad(const float* dY, int rows, float* gb, int cout, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_bgrad_part, dim3(BGRAD_BLOCKS), dim3(256), 0, st, dY, rows, part);
    hipLaunchKernelGGL(k_bgrad_fin, dim3(1), dim3(32), 0, st, part, BGRAD_BLOCKS, gb, cout);
    return hipGetLastError();
}

hipError_t cnn_to_chmajor(const void* in, bool in_f32, unsigned short* out, int rows, hipStream_t st) {
    const int g = (rows + 63) / 64;
    if (in_f32) hipLaunchKernelGGL(k_to_chmajor<true>, dim3(g), dim3(256), 0, st, in, out, rows);
    else hipLaunchKernelGGL(k_to_chmajor<false>, dim3(g), dim3(256), 0, st, in, out, rows);
    return hipGetLastError();
}

hipError_t cnn_f32_to_bf16(const float* in, unsigned short* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

hipError_t cnn_relu_bwd(float* d, const unsigned short* act, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid_for(n)), dim3(256), 0, st, d, act, n);
    return hipGetLastError();
}

hipError_t cnn_w_transpose(const float* w, unsigned short* wt, hipStream_t st) {
    hipLaunchKernelGGL(k_w_transpose, dim3((81 * 1024 + 255) / 256), dim3(256), 0, st, w, wt);
    return hipGetLastError();
}

hipError_t cnn_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                    float c1, float c2, float gscale, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2, gscale);
    return hipGetLastError();
}

hipError_t cnn_half_to_rows(const cd* h, unsigned short* X, const Geom& g, int Ns, const double* scale, int inv,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_half_to_rows, dim3(grid_for((size_t)g.Vh * Ns * 32)), dim3(256), 0, st, h, X, g.Vh, Ns, scale, inv);
    return hipGetLastError();
}

hipError_t cnn_half_to_rows_f32(const cd* h, float* T, const Geom& g, int Ns, const double* scale, hipStream_t st) {
    hipLaunchKernelGGL(k_half_to_rows_f32, dim3(grid_for((size_t)g.Vh * Ns * 32)), dim3(256), 0, st, h, T, g.Vh, Ns, scale);
    return hipGetLastError();
}

hipError_t cnn_rows_to_half(const float* Y, cd* h, const Geom& g, int Ns, const double* scale, hipStream_t st) {
    hipLaunchKernelGGL(k_rows_to_half, dim3(grid_for((size_t)g.Vh * 12 * Ns)), dim3(256), 0, st, Y, h, g.Vh, Ns, scale);
    return hipGetLastError();
}

hipError_t cnn_mse(const float* Y, const float* T, float* dY, size_t n, float w, const Red& red, hipStream_t st) {
    const int grid = grid_for(n);
    hipLaunchKernelGGL(k_mse, dim3(grid), dim3(256), 0, st, Y, T, dY, n, w, red);
    return launch_finish(red, (unsigned)grid, st);
}

}  // namespace eofa
