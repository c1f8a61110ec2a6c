// C ABI of the forcing network (Sec. 2.1, 2.2): model set-up, inference into a
// DG residual, and one Adam training step on the MSE loss.
#include <cmath>
#include <cstring>

#include "nn_internal.hpp"

namespace dgnn {

#define NN_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_error(DG_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                             __FILE__, __LINE__);                                            \
    } while (0)

static int pad32(int x) { return (x + 31) / 32 * 32; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int layout_dims(const int32_t* dims, int32_t n_layers, int* pd, int64_t* n_params, int64_t* n_bf16,
                       int64_t* woff, int64_t* boff, int64_t* wbo, int64_t* wtbo) {
    if (!dims) return set_error(DG_EINVAL, "null dims");
    if (n_layers < 1 || n_layers > kMaxLayers)
        return set_error(DG_EINVAL, "n_layers = %d outside [1, %d]", n_layers, kMaxLayers);
    for (int l = 0; l <= n_layers; ++l) {
        if (dims[l] < 1 || dims[l] > 1024) return set_error(DG_EINVAL, "dims[%d] = %d outside [1, 1024]", l, dims[l]);
        pd[l] = pad32(dims[l]);
    }
    int64_t np = 0, nb = 0;
    for (int l = 0; l < n_layers; ++l) {
        if (woff) woff[l] = np;
        np += (int64_t)dims[l] * dims[l + 1];
        if (boff) boff[l] = np;
        np += dims[l + 1];
        if (wbo) wbo[l] = nb;
        nb += (int64_t)pd[l] * pd[l + 1];
        if (wtbo) wtbo[l] = nb;
        nb += (int64_t)pd[l] * pd[l + 1];
    }
    if (n_params) *n_params = np;
    if (n_bf16) *n_bf16 = nb;
    return DG_OK;
}

NetArgs net_args(const nn_model* m) {
    NetArgs na;
    std::memset(&na, 0, sizeof(na));
    na.n_layers = m->n_layers;
    na.act = m->act;
    for (int l = 0; l <= m->n_layers; ++l) {
        na.dims[l] = m->dims[l];
        na.pdims[l] = m->pdims[l];
    }
    for (int l = 0; l < m->n_layers; ++l) {
        na.W[l] = m->wbf + m->wbf_off[l];
        na.WT[l] = m->wbf + m->wtbf_off[l];
        na.b[l] = m->params + m->boff[l];
    }
    for (int v = 0; v < 5; ++v) {
        na.mu_in[v] = m->norm[v];
        na.sig_in[v] = m->norm[5 + v];
        na.mu_out[v] = m->norm[10 + v];
        na.sig_out[v] = m->norm[15 + v];
        na.mask[v] = m->mask[v];
        na.in_var[v] = m->in_var[v];
        na.out_var[v] = m->out_var[v];
    }
    na.n_in = m->n_in;
    na.n_out = m->n_out;
    na.col = m->col_norm;
    na.col_np = m->col_np;
    return na;
}

int net_check_mesh(const nn_model* m, const Mesh& mesh) {
    if (!m) return set_error(DG_EINVAL, "null model");
    if (m->dims[0] != m->n_in * mesh.n_p || m->dims[m->n_layers] != m->n_out * mesh.n_p)
        return set_error(DG_EINVAL, "network sizes %d -> %d do not match %d and %d variables x %d nodes per element",
                         m->dims[0], m->dims[m->n_layers], m->n_in, m->n_out, mesh.n_p);
    if (m->device != mesh.device) return set_error(DG_EINVAL, "model and mesh live on different devices");
    if (m->col_norm && m->col_np != mesh.n_p)
        return set_error(DG_EINVAL, "per-node normalisation is for %d nodes per element, the mesh has %d", m->col_np,
                         mesh.n_p);
    return DG_OK;
}

int net_forcing_impl(const nn_model* m, const Mesh& mesh, const double* q, double* out, int accumulate,
                     hipStream_t st) {
    const NetArgs na = net_args(m);
    NetTarget tg;
    tg.q = q;
    tg.out = out;
    tg.E = mesh.E;
    tg.blk_begin = 0;
    const int nb = (mesh.E + net_rows_per_block() - 1) / net_rows_per_block();
    if (accumulate) NN_HIP(launch_net_forcing(na, mesh.n_p, &tg, 1, nb, st));
    else NN_HIP(launch_net_forcing_write(na, mesh.n_p, &tg, 1, nb, st));
    return DG_OK;
}

bool grad_net_fusable(const nn_model* m, const Mesh& mesh) {
    // the fused launch pays off once its 16-element blocks fill the GPU (one
    // per CU); on smaller meshes the separate BR1 launch spreads the
    // elements over all CUs and wins
    return m && mesh.PP == 4 && mesh.ph.viscous && mesh.E % net_rows_per_block() == 0 &&
           mesh.E / net_rows_per_block() >= cu_count() && m->dims[0] == m->n_in * mesh.n_p;
}

int grad_net_impl(const nn_model* m, const Mesh& mesh, const DescList& dl, const double* q, double* out,
                  hipStream_t st) {
    const NetArgs na = net_args(m);
    NetTarget tg;
    tg.q = q;
    tg.out = out;
    tg.E = mesh.E;
    tg.blk_begin = 0;
    NN_HIP(launch_grad_net(mesh.PP, dl, na, tg, st));
    return DG_OK;
}

int net_forcing_batch(const nn_model* m, int n_p, const NetTarget* targets, int nt, hipStream_t st) {
    const NetArgs na = net_args(m);
    const int rpb = net_rows_per_block();
    for (int c0 = 0; c0 < nt; c0 += 16) {
        const int cn = nt - c0 < 16 ? nt - c0 : 16;
        NetTarget tg[16];
        int blk = 0;
        for (int i = 0; i < cn; ++i) {
            tg[i] = targets[c0 + i];
            tg[i].blk_begin = blk;
            blk += (tg[i].E + rpb - 1) / rpb;
        }
        NN_HIP(launch_net_forcing_write(na, n_p, tg, cn, blk, st));
    }
    return DG_OK;
}

static int refresh(nn_model* m, hipStream_t st) {
    const NetArgs na = net_args(m);
    for (int l = 0; l < m->n_layers; ++l)
        NN_HIP(launch_net_refresh_layer(na, m->params, m->woff[l], l, m->wbf, m->wbf_off[l], m->wtbf_off[l], st));
    return DG_OK;
}

struct TrainLayout {
    size_t actT[kMaxLayers], dzT[kMaxLayers], part[kMaxLayers], bpart[kMaxLayers], loss, total;
    int Bp, nks, nrb;
};

static TrainLayout train_layout(const nn_model* m, int batch) {
    TrainLayout T;
    std::memset(&T, 0, sizeof(T));
    T.Bp = pad32(batch);
    // the weight-gradient products split the batch into nks slices of at
    // least 256 rows, at most eight (batch 4096: 0.0675 ms per Adam step
    // against 0.071 with sixteen slices, whose partial sums double the
    // traffic of the reduction; 0.0705 with four)
    T.nks = T.Bp / 256;
    if (T.nks < 1) T.nks = 1;
    if (T.nks > 8) T.nks = 8;
    T.nrb = T.Bp / 16;
    size_t off = 0;
    for (int l = 0; l < m->n_layers; ++l) {
        T.actT[l] = off;
        off += align256((size_t)m->pdims[l] * T.Bp * sizeof(uint16_t));
        T.dzT[l] = off;
        off += align256((size_t)m->pdims[l + 1] * T.Bp * sizeof(uint16_t));
        T.part[l] = off;
        off += align256((size_t)T.nks * m->pdims[l] * m->pdims[l + 1] * sizeof(float));
        T.bpart[l] = off;
        off += align256((size_t)T.nrb * m->pdims[l + 1] * sizeof(float));
    }
    T.loss = off;
    off += align256((size_t)(T.Bp / 16 + 1) * sizeof(float));
    T.total = off;
    return T;
}

}  // namespace dgnn

using namespace dgnn;

extern "C" {

int nn_query(const int32_t* dims, int32_t n_layers, int64_t* n_params, int64_t* n_bf16) {
    int pd[kMaxLayers + 1];
    return layout_dims(dims, n_layers, pd, n_params, n_bf16, nullptr, nullptr, nullptr, nullptr);
}

int nn_init(const int32_t* dims, int32_t n_layers, int32_t activation, float* params, uint16_t* w_bf16, float* grad,
            float* adam_m, float* adam_v, const double* norm, const uint8_t* mask, void* stream, nn_model** out) {
    return nn_init_io(dims, n_layers, activation, nullptr, nullptr, params, w_bf16, grad, adam_m, adam_v, norm, mask,
                      stream, out);
}

int nn_init_io(const int32_t* dims, int32_t n_layers, int32_t activation, const uint8_t* in_vars,
               const uint8_t* out_vars, float* params, uint16_t* w_bf16, float* grad, float* adam_m, float* adam_v,
               const double* norm, const uint8_t* mask, void* stream, nn_model** out) {
    if (!out) return set_error(DG_EINVAL, "null output handle");
    *out = nullptr;
    int iv[5], ov[5], n_in = 0, n_out = 0;
    for (int v = 0; v < 5; ++v) {
        if (!in_vars || in_vars[v]) iv[n_in++] = v;
        if (!out_vars || out_vars[v]) ov[n_out++] = v;
    }
    if (n_in == 0 || n_out == 0) return set_error(DG_EINVAL, "the network must read and force at least one variable");
    if (!dims || n_layers < 1 || n_layers > kMaxLayers) return set_error(DG_EINVAL, "bad dims or n_layers");
    if (dims[0] < 1 || dims[n_layers] < 1 || dims[0] % n_in || dims[n_layers] % n_out ||
        dims[0] / n_in != dims[n_layers] / n_out)
        return set_error(DG_EINVAL, "input and output sizes must be %d and %d variables x the same node count", n_in,
                         n_out);
    if (activation != 0 && activation != 1) return set_error(DG_EINVAL, "activation must be 0 (tanh) or 1 (relu)");
    if (!params || !w_bf16 || !norm) return set_error(DG_EINVAL, "null params, bf16 buffer or norm");
    if ((((uintptr_t)params) & 15) || (((uintptr_t)w_bf16) & 255))
        return set_error(DG_EINVAL, "params must be 16-byte and w_bf16 256-byte aligned");
    for (int v = 0; v < 5; ++v)
        if (!(norm[5 + v] > 0) || !(norm[15 + v] > 0) || !std::isfinite(norm[v]) || !std::isfinite(norm[10 + v]))
            return set_error(DG_EINVAL, "normalisation scales must be positive and finite");
    nn_model* m = new nn_model;
    int rc = layout_dims(dims, n_layers, m->pdims, &m->n_params, &m->n_bf16, m->woff, m->boff, m->wbf_off,
                         m->wtbf_off);
    if (rc != DG_OK) {
        delete m;
        return rc;
    }
    m->n_layers = n_layers;
    m->act = activation;
    m->n_in = n_in;
    m->n_out = n_out;
    for (int v = 0; v < 5; ++v) {
        m->in_var[v] = v < n_in ? iv[v] : 0;
        m->out_var[v] = v < n_out ? ov[v] : 0;
    }
    for (int l = 0; l <= n_layers; ++l) m->dims[l] = dims[l];
    m->params = params;
    m->wbf = w_bf16;
    m->grad = grad;
    m->adam_m = adam_m;
    m->adam_v = adam_v;
    std::memcpy(m->norm, norm, sizeof(m->norm));
    for (int v = 0; v < 5; ++v) m->mask[v] = mask ? (mask[v] ? 1.0 : 0.0) : 1.0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete m;
        return set_error(DG_EHIP, "hipGetDevice failed");
    }
    m->device = dev;
    hipStream_t st = (hipStream_t)stream;
    if (adam_m && (rc = (launch_fill_f32(adam_m, 0.0f, m->n_params, st) == hipSuccess ? 0 : DG_EHIP))) {
        delete m;
        return set_error(rc, "zeroing adam_m failed");
    }
    if (adam_v && (rc = (launch_fill_f32(adam_v, 0.0f, m->n_params, st) == hipSuccess ? 0 : DG_EHIP))) {
        delete m;
        return set_error(rc, "zeroing adam_v failed");
    }
    if ((rc = refresh(m, st)) != DG_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return DG_OK;
}

int nn_refresh(nn_model* m, void* stream) {
    if (!m) return set_error(DG_EINVAL, "null model");
    return refresh(m, (hipStream_t)stream);
}

int nn_set_norm(nn_model* m, const double* norm, const uint8_t* mask) {
    if (!m || !norm) return set_error(DG_EINVAL, "null model or norm");
    for (int v = 0; v < 5; ++v)
        if (!(norm[5 + v] > 0) || !(norm[15 + v] > 0)) return set_error(DG_EINVAL, "normalisation scales must be positive");
    std::memcpy(m->norm, norm, sizeof(m->norm));
    if (mask)
        for (int v = 0; v < 5; ++v) m->mask[v] = mask[v] ? 1.0 : 0.0;
    return DG_OK;
}

int nn_set_column_norm(nn_model* m, const double* col_dev, int32_t n_p) {
    if (!m) return set_error(DG_EINVAL, "null model");
    if (!col_dev) {
        m->col_norm = nullptr;
        m->col_np = 0;
        return DG_OK;
    }
    if (n_p < 1 || m->dims[0] != m->n_in * n_p || m->dims[m->n_layers] != m->n_out * n_p)
        return set_error(DG_EINVAL, "n_p = %d does not fit the network sizes", n_p);
    if (((uintptr_t)col_dev) & 7) return set_error(DG_EINVAL, "normalisation array must be 8-byte aligned");
    m->col_norm = col_dev;
    m->col_np = n_p;
    return DG_OK;
}

void nn_free(nn_model* m) { delete m; }

int nn_forcing(const nn_model* m, const dg_mesh* mesh_h, const double* q, double* dqdt, void* ws, size_t ws_bytes,
               void* stream) {
    (void)ws;
    (void)ws_bytes;
    if (!m || !mesh_h) return set_error(DG_EINVAL, "null model or mesh");
    const Mesh& mesh = mesh_h->m;
    int rc = net_check_mesh(m, mesh);
    if (rc) return rc;
    if (!q || !dqdt || q == dqdt) return set_error(DG_EINVAL, "bad field pointers");
    return net_forcing_impl(m, mesh, q, dqdt, 1, (hipStream_t)stream);
}

size_t nn_train_ws(const nn_model* m, int32_t batch) {
    if (!m || batch < 1) return 0;
    return train_layout(m, batch).total;
}

int nn_train_step(nn_model* m, const float* x, const float* y, const int32_t* idx, int32_t batch, float lr,
                  float* loss_dev, void* ws, size_t ws_bytes, void* stream) {
    if (!m) return set_error(DG_EINVAL, "null model");
    if (!m->grad || !m->adam_m || !m->adam_v) return set_error(DG_EINVAL, "model was built without training buffers");
    if (!x || !y || batch < 1) return set_error(DG_EINVAL, "bad batch");
    if (!(lr > 0) || !std::isfinite(lr)) return set_error(DG_EINVAL, "learning rate must be positive");
    if (!ws || (((uintptr_t)ws) & 255)) return set_error(DG_EINVAL, "workspace must be 256-byte aligned");
    const TrainLayout T = train_layout(m, batch);
    if (ws_bytes < T.total) return set_error(DG_ENOSPC, "workspace %zu bytes < %zu needed", ws_bytes, T.total);
    if (train_smem_bytes(net_args(m)) > 160 * 1024 - 2048)
        return set_error(DG_EINVAL, "network too wide for the on-chip training kernel");
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    const NetArgs na = net_args(m);
    TrainArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.x = x;
    ta.y = y;
    ta.idx = idx;
    ta.B = batch;
    ta.Bp = T.Bp;
    ta.grad_scale = (float)(2.0 / ((double)batch * m->dims[m->n_layers]));
    for (int l = 0; l < m->n_layers; ++l) {
        ta.actT[l] = (uint16_t*)(base + T.actT[l]);
        ta.dzT[l] = (uint16_t*)(base + T.dzT[l]);
        ta.bias_part[l] = (float*)(base + T.bpart[l]);
    }
    ta.loss_part = (float*)(base + T.loss);
    const int nblocks = T.nrb;
    NN_HIP(launch_train_rows(na, ta, nblocks, st));
    GradArgs ga;
    std::memset(&ga, 0, sizeof(ga));
    ga.n_layers = m->n_layers;
    ga.Bp = T.Bp;
    ga.nks = T.nks;
    ga.nrb = T.nrb;
    ga.kchunk = ((T.Bp + T.nks - 1) / T.nks + 31) / 32 * 32;
    for (int l = 0; l < m->n_layers; ++l) {
        ga.dzT[l] = ta.dzT[l];
        ga.actT[l] = ta.actT[l];
        ga.part[l] = (float*)(base + T.part[l]);
        ga.bias_part[l] = ta.bias_part[l];
        ga.gW[l] = m->grad + m->woff[l];
        ga.gb[l] = m->grad + m->boff[l];
        ga.pout[l] = m->pdims[l + 1];
        ga.pin[l] = m->pdims[l];
        ga.dout[l] = m->dims[l + 1];
        ga.din[l] = m->dims[l];
        const int ntiles = (ga.pout[l] / 32) * (ga.pin[l] / 32);
        ga.tblk[l + 1] = ga.tblk[l] + (ntiles + 3) / 4;
        ga.rblk[l + 1] = ga.rblk[l] + (ga.dout[l] * ga.din[l] + 255) / 256;
    }
    NN_HIP(launch_wgrad(ga, st));
    m->step += 1;
    const double bc1 = 1.0 - std::pow(0.9, (double)m->step);
    const double bc2 = 1.0 - std::pow(0.999, (double)m->step);
    ParamMap pm;
    std::memset(&pm, 0, sizeof(pm));
    pm.n_layers = m->n_layers;
    for (int l = 0; l < m->n_layers; ++l) {
        pm.woff[l] = m->woff[l];
        pm.boff[l] = m->boff[l];
        pm.wbo[l] = m->wbf_off[l];
        pm.wtbo[l] = m->wtbf_off[l];
        pm.din[l] = m->dims[l];
        pm.dout[l] = m->dims[l + 1];
        pm.pin[l] = m->pdims[l];
        pm.pout[l] = m->pdims[l + 1];
    }
    AdamArgs aa;
    aa.p = m->params;
    aa.m = m->adam_m;
    aa.v = m->adam_v;
    aa.wbf = m->wbf;
    aa.lr = lr;
    aa.b1 = 0.9f;
    aa.b2 = 0.999f;
    aa.eps = 1e-7f;
    aa.bc1 = (float)bc1;
    aa.bc2 = (float)bc2;
    aa.loss_part = ta.loss_part;
    aa.n_loss = nblocks;
    aa.inv_count = (float)(1.0 / ((double)batch * m->dims[m->n_layers]));
    aa.loss = loss_dev;
    NN_HIP(launch_reduce_adam(ga, pm, aa, st));
    return DG_OK;
}

size_t nn_column_stats_ws(int64_t rows, int32_t n_p) {
    if (rows < 1 || n_p < 1) return 0;
    const int nb = (int)(rows < 512 ? rows : 512);
    return align256((size_t)nb * 2 * 5 * n_p * sizeof(double));
}

int nn_column_stats(const float* x, const float* y, int64_t rows, int32_t n_p, double* out_dev, void* ws,
                    size_t ws_bytes, void* stream) {
    if (!x || !y || !out_dev || rows < 1 || n_p < 1) return set_error(DG_EINVAL, "bad arguments");
    if (!ws || (((uintptr_t)ws) & 255)) return set_error(DG_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < nn_column_stats_ws(rows, n_p)) return set_error(DG_ENOSPC, "workspace too small");
    const int nb = (int)(rows < 512 ? rows : 512);
    NN_HIP(launch_column_stats(x, y, rows, 5 * n_p, (double*)ws, nb, out_dev, (hipStream_t)stream));
    return DG_OK;
}

size_t nn_stats_ws(int64_t rows) {
    (void)rows;
    return align256(1024 * 10 * sizeof(double)) + align256(30 * sizeof(double));
}

int nn_data_stats(const float* x, const float* y, int64_t rows, int32_t n_p, double* out_host, void* ws,
                  size_t ws_bytes, void* stream) {
    if (!x || !y || !out_host || rows < 1 || n_p < 1) return set_error(DG_EINVAL, "bad arguments");
    if (!ws || (((uintptr_t)ws) & 255)) return set_error(DG_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < nn_stats_ws(rows)) return set_error(DG_ENOSPC, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    double* part = (double*)ws;
    double* out = (double*)((char*)ws + align256(1024 * 10 * sizeof(double)));
    int nblocks = (int)(rows < 1024 ? rows : 1024);
    NN_HIP(launch_data_stats(x, y, rows, n_p, part, nblocks, out, st));
    NN_HIP(hipMemcpyAsync(out_host, out, 20 * sizeof(double), hipMemcpyDeviceToHost, st));
    NN_HIP(hipStreamSynchronize(st));
    return DG_OK;
}

}  // extern "C"
