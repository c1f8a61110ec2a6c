// Forcing network kernels for gfx950: bf16 MFMA (v_mfma_f32_16x16x32_bf16)
// with float32 accumulation.
//
// Inference (Sec. 2.2, Eq. (4)): one block of sixteen wavefronts takes 16
// elements; their states are gathered from the DG layout q[v][e][n],
// normalised and rounded to bf16 in LDS; every layer is a 16 x N x K product
// of the LDS-resident activations with the bf16 weights read from L2, with
// bias and activation fused into the epilogue; the last layer writes the
// de-normalised forcing straight into the float64 field.  Activations never
// leave LDS.
//
// Training (MSE loss, Adam): the same row blocks run forward, loss and the
// backward data chain with all activations LDS-resident, and write the
// transposed activations and output gradients needed by the weight-gradient
// products dW_l = dz_l^T h_l, which reduce over the batch in a second kernel
// (split over the batch, then a fixed-order sum).
#include "nn_device.hpp"

namespace dgnn {

int net_rows_per_block() { return kRows; }

struct NetTargets {
    NetTarget t[16];
    int n;
};

// ------------------------------------------------------------------ inference

__global__ void __launch_bounds__(kRowThreads) k_net_forcing(NetArgs na, int NP, NetTargets tg, int accumulate) {
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
    int pmax = 0;
    for (int l = 0; l <= na.n_layers; ++l) pmax = pmax > na.pdims[l] ? pmax : na.pdims[l];
    const int ld = pmax + kLdPad;
    uint16_t* bufA = smem;
    uint16_t* bufB = smem + kRows * ld;

    const int b = blockIdx.x;
    int ti = 0;
    for (int i = 1; i < tg.n; ++i)
        if (tg.t[i].blk_begin <= b) ti = i;
    const NetTarget T = tg.t[ti];
    const int e0 = (b - T.blk_begin) * kRows;
    const int E = T.E;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const size_t vs = (size_t)E * NP;

    // gather + normalise + bf16 (zero rows beyond E and columns beyond dims[0])
    const int din = na.dims[0], pin = na.pdims[0];
    for (int idx = t; idx < kRows * pin; idx += kRowThreads) {
        const int r = idx / pin, c = idx - r * pin;
        const int e = e0 + r;
        float x = 0.0f;
        if (e < E && c < din) {
            const int j = c / NP, n = c - j * NP;
            const int v = na.in_var[j];
            x = net_input(na, NP, v, n, gmem(T.q)[v * vs + (size_t)e * NP + n]);
        }
        bufA[r * ld + c] = f2bf(x);
    }
    if (!accumulate) net_zero_unforced(na, NP, T, e0, t);
    __syncthreads();
    net_block_forward(na, NP, T, e0, accumulate, bufA, bufB, ld, wave, lane);
}

// ------------------------------------------------------------------- weights

// bf16 copies of W_l ([pout][pin]) and W_l^T ([pin][pout]), zero padded, in
// the fragment order of wfrag_index
__global__ void __launch_bounds__(256) k_net_refresh(NetArgs na, const float* __restrict__ params,
                                                    uint16_t* __restrict__ wbf,
                                                    int64_t woff0, int l, int64_t wbf_off, int64_t wtbf_off) {
    const int din = na.dims[l], dout = na.dims[l + 1];
    const int pin = na.pdims[l], pout = na.pdims[l + 1];
    const int total = pin * pout;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += gridDim.x * 256) {
        const int o = idx / pin, i = idx - o * pin;
        const float w = (o < dout && i < din) ? params[woff0 + (int64_t)o * din + i] : 0.0f;
        const uint16_t h = f2bf(w);
        wbf[wbf_off + wfrag_index(o, i, pin)] = h;
        wbf[wtbf_off + wfrag_index(i, o, pout)] = h;
    }
}

__global__ void __launch_bounds__(256) k_fill_f32(float* p, float v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = v;
}

// ------------------------------------------------------------------- training

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Columns c < pd of the block's 16 LDS rows (rows r0 .. r0 + 15 of the
// batch) to dst in fragment order over the batch (wfrag_index with K = Bp):
// eight consecutive rows of a column are sixteen contiguous bytes there, so
// each thread packs eight LDS values into one store.
__device__ __forceinline__ void store_transposed(const uint16_t* src, int ld, int pd, global_t<uint16_t>* dst, int r0,
                                                 int Bp, int t) {
    for (int idx = t; idx < pd * 2; idx += kRowThreads) {
        const int c = idx >> 1, g = 8 * (idx & 1);
        u16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = src[(g + j) * ld + c];
        *(global_t<u16x8>*)(dst + wfrag_index(c, r0 + g, Bp)) = v;
    }
}

// One row block: forward with LDS-resident activations, MSE loss in
// normalised space, backward data chain dz_{l-1} = (dz_l W_l) * act'(h_l).
// Writes transposed activations and output gradients for the weight products,
// in fragment order over the batch (wfrag_index with K = Bp).
__global__ void __launch_bounds__(kRowThreads) k_train_rows(NetArgs na, TrainArgs ta) {
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
    const int L = na.n_layers;
    int pmax = 0;
    for (int l = 0; l <= L; ++l) pmax = pmax > na.pdims[l] ? pmax : na.pdims[l];
    const int ld = pmax + kLdPad;
    // act(0..L-1) then two gradient buffers
    auto act = [&](int l) { return smem + l * kRows * ld; };
    uint16_t* g0 = smem + L * kRows * ld;
    uint16_t* g1 = g0 + kRows * ld;
    __shared__ float red[kRowWaves];

    const int r0 = blockIdx.x * kRows;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int B = ta.B, Bp = ta.Bp;
    const int din = na.dims[0], pin = na.pdims[0];
    const int npv_in = din / na.n_in;
    const size_t xw = (size_t)5 * npv_in;
    for (int idx = t; idx < kRows * pin; idx += kRowThreads) {
        const int r = idx / pin, c = idx - r * pin;
        const int row = r0 + r;
        float x = 0.0f;
        if (row < B && c < din) {
            const int j = c / npv_in, n = c - j * npv_in;
            const int v = na.in_var[j];
            const size_t src = ta.idx ? (size_t)ta.idx[row] : (size_t)row;
            const double xv = ta.x[src * xw + (size_t)v * npv_in + n];
            if (na.col) {
                const int cc = v * npv_in + n;
                x = (float)((xv - na.col[cc]) / na.col[5 * npv_in + cc]);
            } else {
                x = (float)((xv - na.mu_in[v]) / na.sig_in[v]);
            }
        }
        act(0)[r * ld + c] = f2bf(x);
    }
    __syncthreads();
    // forward through the hidden layers
    for (int l = 0; l < L - 1; ++l) {
        const int Kp = na.pdims[l], Np = na.pdims[l + 1], Nd = na.dims[l + 1];
        const global_t<const float>* bias = gmem(na.b[l]);
        uint16_t* out = act(l + 1);
        const int a = na.act;
        tile_mma(act(l), ld, gmem(na.W[l]), Kp, Np, wave, lane, [&](int m, int n, float v) {
            const float z = v + (n < Nd ? bias[n] : 0.0f);
            out[m * ld + n] = f2bf(n < Nd ? act_fwd(z, a) : 0.0f);
        });
        __syncthreads();
    }
    // output layer + loss gradient dY = scale (yhat - ytilde)
    float lsum = 0.0f;
    {
        const int l = L - 1;
        const int Kp = na.pdims[l], Np = na.pdims[l + 1], Nd = na.dims[l + 1];
        const int npv_out = Nd / na.n_out;
        const size_t yw = (size_t)5 * npv_out;
        const global_t<const float>* bias = gmem(na.b[l]);
        tile_mma(act(l), ld, gmem(na.W[l]), Kp, Np, wave, lane, [&](int m, int n, float v) {
            const int row = r0 + m;
            float dy = 0.0f;
            if (row < B && n < Nd) {
                const int j = n / npv_out, nn = n - j * npv_out;
                const int vv = na.out_var[j];
                const size_t src = ta.idx ? (size_t)ta.idx[row] : (size_t)row;
                const double yv = ta.y[src * yw + (size_t)vv * npv_out + nn];
                const int cc = vv * npv_out + nn;
                const float yt = na.col ? (float)((yv - na.col[10 * npv_out + cc]) / na.col[15 * npv_out + cc])
                                        : (float)((yv - na.mu_out[vv]) / na.sig_out[vv]);
                const float diff = v + bias[n] - yt;
                lsum += diff * diff;
                dy = ta.grad_scale * diff;
            }
            g0[m * ld + n] = f2bf(dy);
        });
    }
    // the block's loss: a fixed butterfly within each wavefront, then
    // wavefront 0 sums the sixteen partial sums in order (one barrier)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (t == 0) {
        float sum = 0.0f;
        for (int w = 0; w < kRowWaves; ++w) sum += red[w];
        ta.loss_part[blockIdx.x] = sum;
    }
    // row-block sums of dz for the bias gradients (g0 is complete after the barrier above)
    for (int c = t; c < na.pdims[L]; c += kRowThreads) {
        float sacc = 0.0f;
        for (int rr = 0; rr < kRows; ++rr) sacc += bf2f(g0[rr * ld + c]);
        gmem(ta.bias_part[L - 1])[(size_t)blockIdx.x * na.pdims[L] + c] = sacc;
    }
    // transposed activations and dz_{L-1}
    for (int l = 0; l < L; ++l) store_transposed(act(l), ld, na.pdims[l], gmem(ta.actT[l]), r0, Bp, t);
    store_transposed(g0, ld, na.pdims[L], gmem(ta.dzT[L - 1]), r0, Bp, t);
    // backward data chain
    uint16_t* gin = g0;
    uint16_t* gout = g1;
    for (int l = L - 1; l >= 1; --l) {
        const int Kp = na.pdims[l + 1], Np = na.pdims[l], Nd = na.dims[l];
        const uint16_t* h = act(l);
        const int a = na.act;
        tile_mma(gin, ld, gmem(na.WT[l]), Kp, Np, wave, lane, [&](int m, int n, float v) {
            const float d = (n < Nd) ? v * act_bwd(bf2f(h[m * ld + n]), a) : 0.0f;
            gout[m * ld + n] = f2bf(r0 + m < B ? d : 0.0f);
        });
        __syncthreads();
        store_transposed(gout, ld, Np, gmem(ta.dzT[l - 1]), r0, Bp, t);
        for (int c = t; c < Np; c += kRowThreads) {
            float sacc = 0.0f;
            for (int rr = 0; rr < kRows; ++rr) sacc += bf2f(gout[rr * ld + c]);
            gmem(ta.bias_part[l - 1])[(size_t)blockIdx.x * Np + c] = sacc;
        }
        uint16_t* tmp = gin;
        gin = gout;
        gout = tmp;
        __syncthreads();
    }
}

// Weight-gradient partials of every layer in one launch: part_l[ks][o][i] =
// sum over the batch slice ks of dzT_l[o][b] actT_l[i][b].  Each wave computes
// one 32 x 32 tile as 2 x 2 MFMA tiles, so every fragment it loads feeds two
// products; block x (four tiles) belongs to the layer whose block range
// holds it.
__global__ void __launch_bounds__(kThreads) k_wgrad(GradArgs ga) {
    int l = 0;
    while (l + 1 < ga.n_layers && (int)blockIdx.x >= ga.tblk[l + 1]) ++l;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int pout = ga.pout[l], pin = ga.pin[l], Bp = ga.Bp;
    const int tiles_i = pin / 32;
    const int tile = ((int)blockIdx.x - ga.tblk[l]) * 4 + wave;
    const int ntiles = (pout / 32) * tiles_i;
    if (tile >= ntiles) return;
    const int to = tile / tiles_i, tii = tile - to * tiles_i;
    const int ks = blockIdx.y;
    const int kb = ks * ga.kchunk;
    const int ke = kb + ga.kchunk < Bp ? kb + ga.kchunk : Bp;
    const int r = lane & 15;
    // dzT and actT are in fragment order over the batch (wfrag_index with
    // K = Bp): the 32-batch step s of 16-row tile t is the 1 KB block
    // t * Bp / 32 + s, lane-major
    const int ksteps = Bp / 32;
    const global_t<uint16_t>* arow0 = gmem(ga.dzT[l]) + ((int64_t)(2 * to) * ksteps * 64 + lane) * 8;
    const global_t<uint16_t>* arow1 = arow0 + (int64_t)ksteps * 512;
    const global_t<uint16_t>* brow0 = gmem(ga.actT[l]) + ((int64_t)(2 * tii) * ksteps * 64 + lane) * 8;
    const global_t<uint16_t>* brow1 = brow0 + (int64_t)ksteps * 512;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += 32) {
        const int64_t o = (int64_t)(k0 / 32) * 512;
        const bf16x8 a0 = *(const global_t<bf16x8>*)(arow0 + o);
        const bf16x8 a1 = *(const global_t<bf16x8>*)(arow1 + o);
        const bf16x8 b0 = *(const global_t<bf16x8>*)(brow0 + o);
        const bf16x8 b1 = *(const global_t<bf16x8>*)(brow1 + o);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    float* o = ga.part[l] + (size_t)ks * pout * pin;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                o[(size_t)(to * 32 + 16 * i + 4 * (lane >> 4) + v) * pin + tii * 32 + 16 * j + r] = acc[i][j][v];
}

// Adam update of parameter i (flat index) with gradient gi; weights also go
// to their bf16 copies W_l [pout][pin] and W_l^T [pin][pout] (fragment order)
__device__ __forceinline__ void adam_one(const AdamArgs& aa, const ParamMap& pm, int64_t i, float gi) {
    const float mi = aa.b1 * aa.m[i] + (1.0f - aa.b1) * gi;
    const float vi = aa.b2 * aa.v[i] + (1.0f - aa.b2) * gi * gi;
    aa.m[i] = mi;
    aa.v[i] = vi;
    const float pi = aa.p[i] - aa.lr * (mi / aa.bc1) / (sqrtf(vi / aa.bc2) + aa.eps);
    aa.p[i] = pi;
    int l = 0;
    while (l + 1 < pm.n_layers && i >= pm.woff[l + 1]) ++l;
    if (i < pm.boff[l]) {
        const int64_t w = i - pm.woff[l];
        const int o = (int)(w / pm.din[l]), ii = (int)(w - (int64_t)o * pm.din[l]);
        const uint16_t h = f2bf(pi);
        aa.wbf[pm.wbo[l] + wfrag_index(o, ii, pm.pin[l])] = h;
        aa.wbf[pm.wtbo[l] + wfrag_index(ii, o, pm.pout[l])] = h;
    }
}

// The end of a training step in one launch: blocks [0, rblk[L]) sum the
// split-K weight-gradient partials, one thread per weight in a fixed order,
// write the gradient and update that weight (Adam); the next ceil(nbias / 4)
// blocks sum the bias row-block sums, one wavefront per bias (lane-strided
// sums, then a fixed butterfly), and lane 0 updates that bias; with a loss
// output, one more block sums the loss partials.  The same sums in the same
// order as separate reduction launches would make, one launch instead of four.
__global__ void __launch_bounds__(256) k_reduce_adam(GradArgs ga, ParamMap pm, AdamArgs aa, int nbias) {
    const int wblk = ga.rblk[ga.n_layers];
    const int bblk = (nbias + 3) / 4;
    const int b = blockIdx.x;
    if (b < wblk) {
        int l = 0;
        while (l + 1 < ga.n_layers && b >= ga.rblk[l + 1]) ++l;
        const int idx = (b - ga.rblk[l]) * 256 + threadIdx.x;
        const int dout = ga.dout[l], din = ga.din[l], pout = ga.pout[l], pin = ga.pin[l];
        if (idx < dout * din) {
            const int o = idx / din, i = idx - o * din;
            float s = 0.0f;
            for (int k = 0; k < ga.nks; ++k) s += gmem(ga.part[l])[(size_t)k * pout * pin + (size_t)o * pin + i];
            gmem(ga.gW[l])[idx] = s;
            adam_one(aa, pm, pm.woff[l] + idx, s);
        }
        return;
    }
    if (b < wblk + bblk) {
        const int w = (b - wblk) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
        if (w >= nbias) return;
        int l = 0, o = w;
        while (l + 1 < ga.n_layers && o >= ga.dout[l]) {
            o -= ga.dout[l];
            ++l;
        }
        const int pout = ga.pout[l];
        float s = 0.0f;
        for (int k = lane; k < ga.nrb; k += 64) s += gmem(ga.bias_part[l])[(size_t)k * pout + o];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) {
            gmem(ga.gb[l])[o] = s;
            adam_one(aa, pm, pm.boff[l] + o, s);
        }
        return;
    }
    // the loss: sum of the row-block partials
    __shared__ float red[256];
    const int t = threadIdx.x;
    float s = 0.0f;
    for (int i = t; i < aa.n_loss; i += 256) s += aa.loss_part[i];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) aa.loss[0] = red[0] * aa.inv_count;
}

// Per-variable statistics of a training set (rows of 5 n_p floats).  Pass 0
// sums values, pass 1 squared deviations from the pass-0 means; each block
// reduces a contiguous chunk of rows, the final kernel sums the block
// partials in order.
__global__ void __launch_bounds__(256) k_stats_partial(const float* __restrict__ x, const float* __restrict__ y,
                                                      int64_t rows, int n_p, const double* __restrict__ mean,
                                                      double* __restrict__ part) {
    __shared__ double red[10][256];
    const int t = threadIdx.x;
    const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < rows ? r0 + per : rows;
    const int width = 5 * n_p;
    double acc[10];
    for (int c = 0; c < 10; ++c) acc[c] = 0.0;
    for (int64_t r = r0; r < r1; ++r)
        for (int c = t; c < width; c += 256) {
            const int v = c / n_p;
            const double a = x[r * width + c], b = y[r * width + c];
            if (mean) {
                const double da = a - mean[v], db = b - mean[5 + v];
                acc[v] += da * da;
                acc[5 + v] += db * db;
            } else {
                acc[v] += a;
                acc[5 + v] += b;
            }
        }
    for (int c = 0; c < 10; ++c) red[c][t] = acc[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 10; ++c) red[c][t] += red[c][t + w];
        __syncthreads();
    }
    if (t < 10) part[(size_t)blockIdx.x * 10 + t] = red[t][0];
}

__global__ void k_stats_means(const double* __restrict__ out, double* __restrict__ mean) {
    const int c = threadIdx.x;
    if (c < 10) mean[c] = out[10 * (c / 5) + (c % 5)];
}

// out layout: mu_x[5], sigma_x[5], mu_y[5], sigma_y[5]
__global__ void k_stats_final(const double* __restrict__ part, int nblocks, double count, int pass,
                              double* __restrict__ out) {
    const int c = threadIdx.x;
    if (c >= 10) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * 10 + c];
    const int v = c % 5, which = c / 5;          // which: 0 x, 1 y
    if (pass == 0) {
        out[10 * which + v] = s / count;
    } else {
        const double mu = out[10 * which + v];
        const double floor_v = 1e-12 * fmax(1.0, fabs(mu));
        out[10 * which + 5 + v] = fmax(sqrt(s / count), floor_v);
    }
}

// Per-column statistics of a training set (x and y rows of ncols floats):
// block b sums its contiguous chunk of rows for every column (pass 0 values,
// pass 1 squared deviations from the pass-0 means), the final kernel sums the
// block partials in order.  out: [4][ncols] = mu_x, sigma_x, mu_y, sigma_y.
__global__ void __launch_bounds__(256) k_colstats_partial(const float* __restrict__ x, const float* __restrict__ y,
                                                         int64_t rows, int ncols, const double* __restrict__ out,
                                                         int pass, double* __restrict__ part) {
    const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < rows ? r0 + per : rows;
    for (int c = threadIdx.x; c < 2 * ncols; c += 256) {
        const float* A = c < ncols ? x : y;
        const int cc = c < ncols ? c : c - ncols;
        const double mu = pass ? out[(c < ncols ? 0 : 2 * ncols) + cc] : 0.0;
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) {
            const double v = (double)A[r * ncols + cc] - mu;
            s += pass ? v * v : v;
        }
        part[(size_t)blockIdx.x * 2 * ncols + c] = s;
    }
}

__global__ void __launch_bounds__(256) k_colstats_final(const double* __restrict__ part, int nblocks, int ncols,
                                                       double count, int pass, double* __restrict__ out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= 2 * ncols) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * 2 * ncols + c];
    const int base = c < ncols ? 0 : 2 * ncols, cc = c < ncols ? c : c - ncols;
    if (pass == 0) {
        out[base + cc] = s / count;
    } else {
        const double mu = out[base + cc];
        out[base + ncols + cc] = fmax(sqrt(s / count), 1e-12 * fmax(1.0, fabs(mu)));
    }
}

// ------------------------------------------------------------ host launchers

hipError_t launch_data_stats(const float* x, const float* y, int64_t rows, int n_p, double* part, int nblocks,
                             double* out, hipStream_t st) {
    const double count = (double)rows * n_p;
    hipLaunchKernelGGL(k_stats_partial, dim3(nblocks), dim3(256), 0, st, x, y, rows, n_p, (const double*)nullptr,
                       part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, nblocks, count, 0, out);
    // pass 1 needs the means in the layout mean[v] (x) and mean[5 + v] (y): gather them
    hipLaunchKernelGGL(k_stats_means, dim3(1), dim3(64), 0, st, out, out + 20);
    hipLaunchKernelGGL(k_stats_partial, dim3(nblocks), dim3(256), 0, st, x, y, rows, n_p, out + 20, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, nblocks, count, 1, out);
    return hipGetLastError();
}

static size_t net_smem_bytes(const NetArgs& na, int nbuf) {
    int pmax = 0;
    for (int l = 0; l <= na.n_layers; ++l) pmax = pmax > na.pdims[l] ? pmax : na.pdims[l];
    return (size_t)nbuf * kRows * (pmax + kLdPad) * sizeof(uint16_t);
}

hipError_t launch_net_forcing(const NetArgs& na, int n_p, const NetTarget* targets, int nt, int nblocks,
                              hipStream_t st) {
    if (nt < 1 || nt > 16) return hipErrorInvalidValue;
    NetTargets tg;
    for (int i = 0; i < nt; ++i) tg.t[i] = targets[i];
    tg.n = nt;
    const size_t smem = net_smem_bytes(na, 2);
    if (smem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_net_forcing, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_net_forcing, dim3(nblocks), dim3(kRowThreads), smem, st, na, n_p, tg, 1);
    return hipGetLastError();
}

hipError_t launch_net_forcing_write(const NetArgs& na, int n_p, const NetTarget* targets, int nt, int nblocks,
                                    hipStream_t st) {
    if (nt < 1 || nt > 16) return hipErrorInvalidValue;
    NetTargets tg;
    for (int i = 0; i < nt; ++i) tg.t[i] = targets[i];
    tg.n = nt;
    const size_t smem = net_smem_bytes(na, 2);
    if (smem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_net_forcing, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_net_forcing, dim3(nblocks), dim3(kRowThreads), smem, st, na, n_p, tg, 0);
    return hipGetLastError();
}

hipError_t launch_net_refresh_layer(const NetArgs& na, const float* params, int64_t woff, int l, uint16_t* wbf,
                                    int64_t wbf_off, int64_t wtbf_off, hipStream_t st) {
    const int total = na.pdims[l] * na.pdims[l + 1];
    int blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_net_refresh, dim3(blocks), dim3(256), 0, st, na, params, wbf, woff, l, wbf_off,
                       wtbf_off);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, size_t n, hipStream_t st) {
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

size_t train_smem_bytes(const NetArgs& na) { return net_smem_bytes(na, na.n_layers + 2); }

hipError_t launch_train_rows(const NetArgs& na, const TrainArgs& ta, int nblocks, hipStream_t st) {
    const size_t smem = train_smem_bytes(na);
    if (smem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_train_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_train_rows, dim3(nblocks), dim3(kRowThreads), train_smem_bytes(na), st, na, ta);
    return hipGetLastError();
}

hipError_t launch_wgrad(const GradArgs& ga, hipStream_t st) {
    hipLaunchKernelGGL(k_wgrad, dim3(ga.tblk[ga.n_layers], ga.nks), dim3(kThreads), 0, st, ga);
    return hipGetLastError();
}

hipError_t launch_reduce_adam(const GradArgs& ga, const ParamMap& pm, const AdamArgs& aa, hipStream_t st) {
    int nbias = 0;
    for (int l = 0; l < ga.n_layers; ++l) nbias += ga.dout[l];
    const int blocks = ga.rblk[ga.n_layers] + (nbias + 3) / 4 + (aa.loss ? 1 : 0);
    hipLaunchKernelGGL(k_reduce_adam, dim3(blocks), dim3(256), 0, st, ga, pm, aa, nbias);
    return hipGetLastError();
}

hipError_t launch_column_stats(const float* x, const float* y, int64_t rows, int ncols, double* part, int nblocks,
                               double* out, hipStream_t st) {
    const int fb = (2 * ncols + 255) / 256;
    const double count = (double)rows;
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_colstats_partial, dim3(nblocks), dim3(256), 0, st, x, y, rows, ncols,
                           (const double*)out, pass, part);
        hipLaunchKernelGGL(k_colstats_final, dim3(fb), dim3(256), 0, st, part, nblocks, ncols, count, pass, out);
    }
    return hipGetLastError();
}

}  // namespace dgnn
