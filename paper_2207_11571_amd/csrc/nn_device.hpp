// Device code of the forcing network shared by the network kernels and the
// fused BR1-and-network kernel of the stage: bf16 rounding, activations, the
// 16-row MFMA layer product (v_mfma_f32_16x16x32_bf16, float32
// accumulation) and the forward pass of one 16-row block whose normalised
// inputs are in LDS.
#pragma once

#include "dgnn_internal.hpp"

namespace dgnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Global-memory views of pointers taken from the argument structs: indexed
// by a run-time layer number they reach the kernel as generic pointers, and
// generic (flat) accesses count against the LDS counter as well, so LDS
// accesses would wait for the global traffic in flight.
template <class T>
using global_t = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ global_t<T>* gmem(T* p) { return (global_t<T>*)p; }

constexpr int kRows = 16;      // rows (elements / samples) per block
constexpr int kThreads = 256;     // weight-gradient blocks: four wavefronts, one tile each
constexpr int kRowWaves = 16;     // row-block kernels: sixteen wavefronts share the column tiles
constexpr int kRowThreads = 64 * kRowWaves;
constexpr int kLdPad = 8;      // LDS row padding (bf16 elements)

// Weight fragments are read with buffer loads through a resource over one
// layer's bf16 weights [Np][Kp]: one vector offset per lane, the 1 KB steps
// of a tile as scalar offsets.  Plain global loads need an address register
// of their own for every step past the 4 KB immediate offset.
constexpr int kBufferWord3 = 0x00020000;   // fourth resource word, gfx9 family (32-bit data format)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t weight_rsrc(const __attribute__((address_space(1))) uint16_t* W,
                                                               int Kp, int Np) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(const uint16_t*)W, 0, Np * Kp * 2, kBufferWord3);
}

// fragment step s of the tile whose lane offset (bytes) is vo
__device__ __forceinline__ bf16x8 weight_frag(__amdgpu_buffer_rsrc_t rs, int vo, int s) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, s * 1024, 0));
}

// float32 -> bfloat16, round to nearest even (NaN kept quiet); a select,
// not a branch, for the NaN case
__device__ __forceinline__ uint16_t f2bf(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    const uint32_t qnan = (u >> 16) | 0x0040u;
    return (uint16_t)((u & 0x7FFFFFFFu) > 0x7F800000u ? qnan : r);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ float act_fwd(float z, int act) { return act == 0 ? tanhf(z) : fmaxf(z, 0.0f); }
// derivative through the output h = act(z)
__device__ __forceinline__ float act_bwd(float h, int act) { return act == 0 ? 1.0f - h * h : (h > 0.0f ? 1.0f : 0.0f); }

// Position of W[n][k] (n < Np, k < Kp, both padded to multiples of 32) in
// the bf16 weight copies: the fragment order of the B operand of
// v_mfma_f32_16x16x32_bf16 as tile_mma loads it.  Each 16-column tile and
// 32-wide K step is one 1 KB block in which lane r + 16 q holds
// W[16 tile + r][32 s + 8 q, + 8), so that a wavefront's fragment load reads
// one contiguous kilobyte instead of 64-byte pieces of sixteen rows (half
// the time of a row-major layout for the chain of layers, measured).
__host__ __device__ __forceinline__ int64_t wfrag_index(int n, int k, int Kp) {
    const int tile = n >> 4, r = n & 15, s = k >> 5, q = (k & 31) >> 3, j = k & 7;
    return ((((int64_t)tile * (Kp >> 5) + s) * 64 + r + 16 * q) << 3) + j;
}

// C[16][Np] = A[16][Kp] W^T with W [Np][Kp] bf16 in global memory, in the
// fragment order of wfrag_index.
// Wave w computes the 16-column tiles w, w + kRowWaves, ...; epi(m, n, value)
// per output.  For the common widths the K loop is unrolled so that all of a
// tile's weight fragments are in flight at once: the weights come from L2 and
// their latency, not the matrix cores, bounds this product, so sixteen
// wavefronts (one or two tiles each) beat fewer wavefronts with prefetching.
template <int KP, class Epi>
__device__ __forceinline__ void tile_mma_fixed(const uint16_t* __restrict__ sA, int ldA,
                                               const global_t<uint16_t>* __restrict__ W, int Np, int wave, int lane,
                                               Epi& epi) {
    constexpr int KS = KP / 32;
    const int kq = 8 * (lane >> 4);
    const int r = lane & 15;
    const uint16_t* arow = sA + r * ldA + kq;
    const __amdgpu_buffer_rsrc_t rs = weight_rsrc(W, KP, Np);
    for (int tile = wave; tile < Np / 16; tile += kRowWaves) {
        const int vo = (tile * KS * 64 + lane) * 16;
        bf16x8 b[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) b[s] = weight_frag(rs, vo, s);
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const bf16x8 a = *(const bf16x8*)(arow + 32 * s);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[s], acc, 0, 0, 0);
        }
        const int n = tile * 16 + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) epi(4 * (lane >> 4) + i, n, acc[i]);
    }
}

template <class Epi>
__device__ __forceinline__ void tile_mma(const uint16_t* __restrict__ sA, int ldA,
                                         const global_t<uint16_t>* __restrict__ W, int Kp, int Np, int wave, int lane,
                                         Epi epi) {
    if (Kp == 256) {
        tile_mma_fixed<256>(sA, ldA, W, Np, wave, lane, epi);
        return;
    }
    if (Kp == 320) {
        tile_mma_fixed<320>(sA, ldA, W, Np, wave, lane, epi);
        return;
    }
    const int kq = 8 * (lane >> 4);
    const int r = lane & 15;
    for (int tile = wave; tile < Np / 16; tile += kRowWaves) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        const int n = tile * 16 + r;
        const global_t<uint16_t>* wt = W + ((int64_t)tile * (Kp / 32) * 64 + lane) * 8;
        const uint16_t* arow = sA + r * ldA + kq;
        for (int k0 = 0; k0 < Kp; k0 += 32) {
            const bf16x8 a = *(const bf16x8*)(arow + k0);
            const bf16x8 b = *(const global_t<bf16x8>*)(wt + (k0 / 32) * 512);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) epi(4 * (lane >> 4) + i, n, acc[i]);
    }
}

// Layers with K <= 32 * kMaxKS = 320 keep a wavefront's whole weight tile in
// registers, so the next layer's tile can be loaded while the current one's
// outputs are formed (below).
constexpr int kMaxKS = 10;

// issue the loads of this wavefront's fragments of column tile `tile` of W
// [Np][Kp].  (Each load sits under its own branch, the count being known at
// run time; with global loads and their per-step address registers the
// compiler waited for all loads in flight before each step past the first
// four, which the buffer loads avoid.)
__device__ __forceinline__ void load_frags(bf16x8 (&b)[kMaxKS], const global_t<uint16_t>* W, int Kp, int Np, int tile,
                                           int lane) {
    const int KS = Kp >> 5;
    const __amdgpu_buffer_rsrc_t rs = weight_rsrc(W, Kp, Np);
    const int vo = (tile * KS * 64 + lane) * 16;
#pragma unroll
    for (int s = 0; s < kMaxKS; ++s)
        if (s < KS) b[s] = weight_frag(rs, vo, s);
}

// C tile = A[16][Kp] (LDS rows from arow) times the fragments b
__device__ __forceinline__ floatx4 mma_frags(const bf16x8 (&b)[kMaxKS], const uint16_t* arow, int Kp) {
    const int KS = Kp >> 5;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < kMaxKS; ++s)
        if (s < KS) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8*)(arow + 32 * s), b[s], acc, 0, 0, 0);
    return acc;
}

// normalised network input of node n of variable v, value qv (Sec. 2.2:
// per-variable, or per-node when the model carries column statistics)
__device__ __forceinline__ float net_input(const NetArgs& na, int NP, int v, int n, double qv) {
    if (na.col) {
        const int cc = v * NP + n;
        return (float)((qv - na.col[cc]) / na.col[5 * NP + cc]);
    }
    return (float)((qv - na.mu_in[v]) / na.sig_in[v]);
}

// write mode: the variables the network does not force get s = 0 (rows
// e0 .. e0 + 15 of target T)
__device__ __forceinline__ void net_zero_unforced(const NetArgs& na, int NP, const NetTarget& T, int e0, int t) {
    if (na.n_out >= 5) return;
    const size_t vs = (size_t)T.E * NP;
    for (int idx = t; idx < kRows * 5 * NP; idx += kRowThreads) {
        const int r = idx / (5 * NP), c = idx - r * (5 * NP);
        const int v = c / NP, n = c - v * NP;
        const int e = e0 + r;
        bool forced = false;
        for (int j = 0; j < na.n_out; ++j) forced = forced || na.out_var[j] == v;
        if (e < T.E && !forced) gmem(T.out)[v * vs + (size_t)e * NP + n] = 0.0;
    }
}

// The layers of one 16-row block: bufA holds the rows' normalised bf16
// inputs (zero beyond dims[0] and for rows past the target's end), bufB is
// scratch of the same shape; hidden layers apply bias and activation, the
// last layer de-normalises and writes (or adds) s for rows e0 .. e0 + 15 of
// T.  Ends with a block barrier.
__device__ __forceinline__ void net_block_forward(const NetArgs& na, int NP, const NetTarget& T, int e0, int accumulate,
                                                  uint16_t* bufA, uint16_t* bufB, int ld, int wave, int lane) {
    const size_t vs = (size_t)T.E * NP;
    const int L = na.n_layers;
    // Narrow layers: each wavefront's weight tile of the next layer is
    // loaded as soon as the products of its last tile of this layer are
    // issued, so the load latency overlaps the bias / activation epilogue
    // and the block barrier instead of starting after them.
    bool narrow = true;
    for (int l = 0; l < L; ++l) narrow = narrow && na.pdims[l] <= 32 * kMaxKS;
    if (narrow) {
        const int r = lane & 15;
        const int kq = 8 * (lane >> 4);
        bf16x8 b[kMaxKS];
        if (wave < na.pdims[1] / 16) load_frags(b, gmem(na.W[0]), na.pdims[0], na.pdims[1], wave, lane);
        for (int l = 0; l < L; ++l) {
            const int Kp = na.pdims[l], Np = na.pdims[l + 1], Nd = na.dims[l + 1];
            const global_t<const float>* bias = gmem(na.b[l]);
            const uint16_t* arow = bufA + r * ld + kq;
            // a wavefront with no tile in this layer but one in the next
            if (l + 1 < L && wave >= Np / 16 && wave < na.pdims[l + 2] / 16)
                load_frags(b, gmem(na.W[l + 1]), Np, na.pdims[l + 2], wave, lane);
            for (int tile = wave; tile < Np / 16; tile += kRowWaves) {
                if (tile != wave) load_frags(b, gmem(na.W[l]), Kp, Np, tile, lane);
                const floatx4 acc = mma_frags(b, arow, Kp);
                if (tile + kRowWaves >= Np / 16 && l + 1 < L && wave < na.pdims[l + 2] / 16)
                    load_frags(b, gmem(na.W[l + 1]), Np, na.pdims[l + 2], wave, lane);
                const int n = tile * 16 + r;
                if (l < L - 1) {
                    const float bn = n < Nd ? bias[n] : 0.0f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int m = 4 * (lane >> 4) + i;
                        bufB[m * ld + n] = f2bf(n < Nd ? act_fwd(acc[i] + bn, na.act) : 0.0f);
                    }
                } else if (n < Nd) {
                    const float bn = bias[n];
                    const int j = n / NP, node = n - j * NP;
                    const int vv = na.out_var[j];
                    const int cc = vv * NP + node;
                    const double sc = na.col ? na.mask[vv] * na.col[15 * NP + cc] : na.mask[vv] * na.sig_out[vv];
                    const double sh = na.col ? na.mask[vv] * na.col[10 * NP + cc] : na.mask[vv] * na.mu_out[vv];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int e = e0 + 4 * (lane >> 4) + i;
                        if (e < T.E) {
                            const double s = sc * (double)(acc[i] + bn) + sh;
                            global_t<double>* o = gmem(T.out) + vv * vs + (size_t)e * NP + node;
                            *o = accumulate ? *o + s : s;
                        }
                    }
                }
            }
            __syncthreads();
            uint16_t* tmp = bufA;
            bufA = bufB;
            bufB = tmp;
        }
        return;
    }
    for (int l = 0; l < L; ++l) {
        const int Kp = na.pdims[l], Np = na.pdims[l + 1], Nd = na.dims[l + 1];
        const global_t<const float>* bias = gmem(na.b[l]);
        if (l < L - 1) {
            const int act = na.act;
            tile_mma(bufA, ld, gmem(na.W[l]), Kp, Np, wave, lane, [&](int m, int n, float v) {
                const float z = v + (n < Nd ? bias[n] : 0.0f);
                bufB[m * ld + n] = f2bf(n < Nd ? act_fwd(z, act) : 0.0f);
            });
        } else {
            tile_mma(bufA, ld, gmem(na.W[l]), Kp, Np, wave, lane, [&](int m, int n, float v) {
                const int e = e0 + m;
                if (e < T.E && n < Nd) {
                    const float y = v + bias[n];
                    const int j = n / NP, node = n - j * NP;
                    const int vv = na.out_var[j];
                    const int cc = vv * NP + node;
                    const double s = na.col ? na.mask[vv] * (na.col[15 * NP + cc] * (double)y + na.col[10 * NP + cc])
                                            : na.mask[vv] * (na.sig_out[vv] * (double)y + na.mu_out[vv]);
                    global_t<double>* o = gmem(T.out) + vv * vs + (size_t)e * NP + node;
                    *o = accumulate ? *o + s : s;
                }
            });
        }
        __syncthreads();
        uint16_t* tmp = bufA;
        bufA = bufB;
        bufB = tmp;
    }
}

}  // namespace dgnn
