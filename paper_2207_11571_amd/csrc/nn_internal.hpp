// Internal side of the forcing network: the model object and the entry
// points the DG stepping and the server call.  Not part of the public ABI.
#pragma once

#include "dgnn_internal.hpp"

struct nn_model {
    int n_layers = 0;
    int act = 0;
    int dims[dgnn::kMaxLayers + 1] = {0};
    int pdims[dgnn::kMaxLayers + 1] = {0};
    float* params = nullptr;      // caller-owned, float32 master
    uint16_t* wbf = nullptr;      // caller-owned, bf16 copies (W then W^T per layer)
    float* grad = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int64_t n_params = 0, n_bf16 = 0;
    int64_t woff[dgnn::kMaxLayers] = {0};    // W_l offset in params
    int64_t boff[dgnn::kMaxLayers] = {0};    // b_l offset in params
    int64_t wbf_off[dgnn::kMaxLayers] = {0}; // W_l offset in wbf
    int64_t wtbf_off[dgnn::kMaxLayers] = {0};// W_l^T offset in wbf
    double norm[20] = {0};
    double mask[5] = {1, 1, 1, 1, 1};
    int n_in = 5, n_out = 5;                 // variables read / forced
    int in_var[5] = {0, 1, 2, 3, 4};
    int out_var[5] = {0, 1, 2, 3, 4};
    const double* col_norm = nullptr;        // per-node normalisation (device, caller-owned) or null
    int col_np = 0;
    int64_t step = 0;                        // Adam step counter
    int device = 0;
};

namespace dgnn {

NetArgs net_args(const nn_model* m);
int net_check_mesh(const nn_model* m, const Mesh& mesh);
// out = s(q) (accumulate == 0) or out += s(q), for one mesh-sized field
int net_forcing_impl(const nn_model* m, const Mesh& mesh, const double* q, double* out, int accumulate,
                     hipStream_t st);
// batched: several solves' fields in one launch (all on meshes of the same order)
int net_forcing_batch(const nn_model* m, int n_p, const NetTarget* targets, int nt, hipStream_t st);
// whether the stage's BR1 pass and the network (write mode, out = s(q)) can
// run as one launch (launch_grad_net) on this mesh
bool grad_net_fusable(const nn_model* m, const Mesh& mesh);
// the BR1 pass of the stage described by dl and out = s(q) in one launch
int grad_net_impl(const nn_model* m, const Mesh& mesh, const DescList& dl, const double* q, double* out,
                  hipStream_t st);

}  // namespace dgnn
