// Internal declarations shared by the HIP kernels (kernels.hip) and the host
// side of the library (api.cpp, server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/dgnn.h"

namespace dgnn {

constexpr int kMaxPP = DG_MAX_ORDER + 1;   // nodes per direction at the highest order
constexpr int kMaxLayers = 8;               // weight layers of the forcing network
constexpr int kMaxDevices = 64;             // GPUs a process can build meshes on

// Gauss-Legendre nodal basis of one order (Sec. 2.6).  D[i*PP + j] = l_j'(xi_i);
// Dhat[i*PP + m] = D[m][i] w_m / w_i is the weak-form volume operator;
// bpw = b+/w and bmw = b-/w lift interface values into the volume.
struct BasisTab {
    double nodes[kMaxPP];
    double w[kMaxPP];
    double D[kMaxPP * kMaxPP];
    double Dhat[kMaxPP * kMaxPP];
    double bp[kMaxPP];
    double bm[kMaxPP];
    double bpw[kMaxPP];
    double bmw[kMaxPP];
    // the weak derivative along a line evaluated at the line's minus (0) and
    // plus (1) end: dface[s][l] = sum_m b_s(m) Dhat[m][l] and the lifting
    // weights lface_p[s] = sum_m b_s(m) b+_m/w_m, lface_m[s] = sum_m b_s(m) b-_m/w_m
    double dface[2][kMaxPP];
    double lface_p[2];
    double lface_m[2];
};

// Per-solve physical constants, in the form the kernels use them.
struct Phys {
    double gamma, gm1;      // gamma, gamma - 1
    double p_ref;           // subtracted from the momentum fluxes
    double mu, kappa;       // molecular viscosity and conductivity
    double les_c;           // (Cs * h / (P + 1))^2, 0 without the closure
    double kt;              // gamma / ((gamma - 1) Pr_t): mu_t -> kappa_t
    double s;               // 2 / h: d/dx = s d/dxi
    double h, L;            // element size and box side
    double p0;              // background pressure of the TGV state
    int viscous;            // BR1 gradients and viscous fluxes
    int les;                // Smagorinsky closure
};

// One solve as the batched stage kernels see it (device memory).
struct SolveDesc {
    double* q;              // state [5][E][n_p]
    double* k;              // Runge-Kutta register [5][E][n_p]
    double* out;            // residual output [5][E][n_p] (residual mode)
    const double* forcing;  // s(q) [5][E][n_p] added to the residual, or null
    const double* post;     // update mode: q += dt post after the stage update
                            // (a post-step correction), or null
    const double* qtr_in;   // face traces of q   [E][6][5][n_f]
    double* qtr_out;        // face traces of the updated q (update mode)
    double* fv;             // one-sided viscous normal fluxes [E][6][4][n_f]
    int N, E;
    double dt;
    Phys ph;
};

// The solves one stage launch works on (by value, in the kernel arguments):
// blocks [blk[i], blk[i+1]) work on *d[i], one element per block.
constexpr int kMaxDescs = 32;
struct DescList {
    const SolveDesc* d[kMaxDescs];
    int blk[kMaxDescs + 1];
    int n;
    // one solve whose descriptor the host also has: a copy travels in the
    // kernel arguments (inl = 1), so the stage kernels read its fields
    // there instead of through the pointer (two dependent loads fewer
    // before a block's first data load)
    int inl;
    SolveDesc d0;
};

// Forcing-network description passed by value to the network kernels.
struct NetArgs {
    int n_layers;
    int act;                         // 0 tanh, 1 relu
    int dims[kMaxLayers + 1];        // true sizes
    int pdims[kMaxLayers + 1];       // sizes rounded up to 32
    const uint16_t* W[kMaxLayers];   // bf16 [pdims[l+1]][pdims[l]], zero padded
    const uint16_t* WT[kMaxLayers];  // bf16 [pdims[l]][pdims[l+1]], zero padded
    const float* b[kMaxLayers];      // float32 [dims[l+1]]
    double mu_in[5], sig_in[5], mu_out[5], sig_out[5], mask[5];
    // the network reads variables in_var[0..n_in) (input column j n_p + n is
    // node n of variable in_var[j]) and forces out_var[0..n_out) likewise
    int n_in, n_out;
    int in_var[5], out_var[5];
    // per-node normalisation (null: per variable): device [4][5 col_np] doubles,
    // mu_in, sigma_in, mu_out, sigma_out of row column v col_np + n
    const double* col;
    int col_np;
};

// One network application target for the batched forcing kernel: the
// elements of one solve, in blocks of rows.
struct NetTarget {
    const double* q;        // [5][E][n_p]
    double* out;            // [5][E][n_p], out += s(q)
    int E;
    int blk_begin;
};

struct Mesh {
    dg_params prm;
    int N, P, PP, E, n_p, n_f;
    Phys ph;
    int device;
};

}  // namespace dgnn

struct dg_mesh {
    dgnn::Mesh m;
};

namespace dgnn {

// workspace layout of one mesh, in bytes from the workspace base
struct WsLayout {
    size_t desc, qtr0, qtr1, fv, forcing, partial, total;
};
WsLayout ws_layout(const Mesh& m);

void fill_phys(const dg_params& p, Phys& ph);

// ----------------------------------------------------------- host launchers
// All return hipSuccess or the launch error.  `descs` is device memory.
hipError_t upload_basis_tables(const BasisTab* host_tabs /* index P-1 */);
// address of the no-alloc stepper's scratch on device dev (looked up once, by
// scratch_setup with dev current); null before the set-up
hipError_t scratch_setup(int dev);
void* scratch_device_ptr(int dev);
hipError_t launch_write_descs(const SolveDesc* host, int n, SolveDesc* dev, hipStream_t st);
hipError_t launch_traces(int PP, const DescList& dl, hipStream_t st);
// compute units of the current device
int cu_count();
hipError_t launch_grad(int PP, const DescList& dl, hipStream_t st);
// k_grad and the forcing network in one launch (P = 3, one solve, E a
// multiple of 16, the network reading all n_p nodes of its variables);
// hipErrorInvalidValue otherwise
hipError_t launch_grad_net(int PP, const DescList& dl, const NetArgs& na, const NetTarget& T, hipStream_t st);
hipError_t launch_resid(int PP, int update, const DescList& dl, double rkA, double rkB, int first_stage,
                        hipStream_t st);
hipError_t launch_tgv(int PP, const Phys& ph, int N, double* q, hipStream_t st);
hipError_t launch_diag(int PP, const Phys& ph, int N, const double* q, double* partial,
                       double* out, hipStream_t st);
hipError_t launch_err_inf(int PP, int E, const double* q, const double* qref, double* partial,
                          double* out, hipStream_t st);
hipError_t launch_project(int PPs, int PPd, int E, const double* G1 /* host [PPd][PPs] */,
                          const double* src, double* dst, hipStream_t st);
hipError_t launch_pack_pairs(int E, int n_p, double div, const double* Gq, const double* GR, const double* R3,
                             float* x, float* y, hipStream_t st);

hipError_t launch_net_forcing(const NetArgs& na, int n_p, const NetTarget* targets, int nt,
                              int nblocks, hipStream_t st);             // out += s(q)
hipError_t launch_net_forcing_write(const NetArgs& na, int n_p, const NetTarget* targets, int nt,
                                    int nblocks, hipStream_t st);       // out = s(q)
hipError_t launch_net_refresh_layer(const NetArgs& na, const float* params, int64_t woff, int l,
                                    uint16_t* wbf, int64_t wbf_off, int64_t wtbf_off, hipStream_t st);
hipError_t launch_fill_f32(float* p, float v, size_t n, hipStream_t st);
int net_rows_per_block();

// training: per-row-block forward / loss / backward data chain, then the
// weight-gradient products reduced over the batch, then Adam
struct TrainArgs {
    const float* x;                   // [rows][5 n_p] (all variables)
    const float* y;                   // [rows][5 n_p]
    const int32_t* idx;               // batch row b is row idx[b] (null: row b)
    int B, Bp;                        // batch, batch rounded up to 32
    float grad_scale;                 // 2 / (B * dims[L])
    uint16_t* actT[kMaxLayers];       // [pdims[l]][Bp]  (act[0] = xhat)
    uint16_t* dzT[kMaxLayers];        // [pdims[l+1]][Bp]
    float* bias_part[kMaxLayers];     // [Bp / 16][pdims[l+1]] row-block sums of dz_l
    float* loss_part;                 // [Bp / 16]
};

// All layers' weight and bias gradients of one training step: split-K
// partial products, then one fixed-order reduction.
struct GradArgs {
    const uint16_t* dzT[kMaxLayers];
    const uint16_t* actT[kMaxLayers];
    float* part[kMaxLayers];          // [nks][pout][pin]
    const float* bias_part[kMaxLayers];
    float* gW[kMaxLayers];
    float* gb[kMaxLayers];
    int pout[kMaxLayers], pin[kMaxLayers], dout[kMaxLayers], din[kMaxLayers];
    int tblk[kMaxLayers + 1];         // product blocks before layer l (four 16x16 tiles each)
    int rblk[kMaxLayers + 1];         // reduction blocks before layer l (256 outputs each)
    int n_layers, Bp, kchunk, nks, nrb;
};

// Adam on the float32 master weights with the bf16 copies W_l, W_l^T written
// in the same pass.
struct ParamMap {
    int64_t woff[kMaxLayers], boff[kMaxLayers], wbo[kMaxLayers], wtbo[kMaxLayers];
    int din[kMaxLayers], dout[kMaxLayers], pin[kMaxLayers], pout[kMaxLayers];
    int n_layers;
};
// Adam step of the whole parameter vector (and the loss output, when loss is
// not null), for the fused end-of-step launch
struct AdamArgs {
    float* p;
    float* m;
    float* v;
    uint16_t* wbf;
    float lr, b1, b2, eps, bc1, bc2;
    const float* loss_part;
    int n_loss;
    float inv_count;
    float* loss;
};
size_t train_smem_bytes(const NetArgs& na);
hipError_t launch_train_rows(const NetArgs& na, const TrainArgs& ta, int nblocks, hipStream_t st);
// the split-K weight-gradient products alone, and then the gradient
// reductions, the Adam update and the loss in one launch
hipError_t launch_wgrad(const GradArgs& ga, hipStream_t st);
hipError_t launch_reduce_adam(const GradArgs& ga, const ParamMap& pm, const AdamArgs& aa, hipStream_t st);
hipError_t launch_data_stats(const float* x, const float* y, int64_t rows, int n_p, double* part, int nblocks,
                             double* out_dev, hipStream_t st);
hipError_t launch_column_stats(const float* x, const float* y, int64_t rows, int ncols, double* part, int nblocks,
                               double* out_dev, hipStream_t st);

// error reporting (thread-local)
int set_error(int code, const char* fmt, ...);

// host-side building blocks shared by the C ABI and the solve server
extern const double kRkA[3];
extern const double kRkB[3];
int make_mesh(const dg_params* prm, Mesh& M);
DescList single_list(const SolveDesc* d, int E);
// the same with the host's copy of the descriptor carried along
DescList single_list(const SolveDesc* d, const SolveDesc& host, int E);
int residual_impl(const Mesh& m, const double* q, double* dqdt, char* ws, hipStream_t st);
int diag_impl(const Mesh& m, const double* q, double* out_dev, char* ws, hipStream_t st);
int project_impl(const Mesh& src, const Mesh& dst, const double* f_src, double* f_dst, hipStream_t st);
int init_tgv_impl(const Mesh& m, double* q, hipStream_t st);
double stable_dt_from_diag(const Mesh& m, const double* diag_host, double cfl);

}  // namespace dgnn
