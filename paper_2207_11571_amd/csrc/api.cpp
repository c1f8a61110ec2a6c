// C ABI of the DG part of libdgnn: mesh set-up (host basis tables), residual,
// Runge-Kutta stepping, diagnostics, filter G and training-pair generation.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dgnn_internal.hpp"
#include "nn_internal.hpp"

namespace dgnn {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define DG_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_error(DG_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                             __FILE__, __LINE__);                                            \
    } while (0)

// ------------------------------------------------------------ host basis

// Legendre polynomial L_n and derivative by the three-term recurrence (long double)
static void legendre_ld(int n, long double x, long double& L, long double& dL) {
    long double p0 = 1.0L, p1 = x;
    if (n == 0) { L = 1.0L; dL = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    L = p1;
    dL = n * (x * p1 - p0) / (x * x - 1.0L);
}

// Gauss-Legendre points/weights (Newton on L_{P+1}), barycentric Lagrange
// differentiation and boundary interpolation, in long double, rounded once.
static void host_basis(int P, BasisTab& T) {
    const int n = P + 1;
    std::memset(&T, 0, sizeof(T));
    long double x[kMaxPP], w[kMaxPP], lam[kMaxPP];
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double xi = -cosl(pi * (i + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double L, dL;
            legendre_ld(n, xi, L, dL);
            long double dx = L / dL;
            xi -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        long double L, dL;
        legendre_ld(n, xi, L, dL);
        x[i] = xi;
        w[i] = 2.0L / ((1.0L - xi * xi) * dL * dL);
    }
    for (int j = 0; j < n; ++j) {
        long double p = 1.0L;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (x[j] - x[k]);
        lam[j] = 1.0L / p;
    }
    long double D[kMaxPP][kMaxPP];
    for (int i = 0; i < n; ++i) {
        long double diag = 0.0L;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i][j] = (lam[j] / lam[i]) / (x[i] - x[j]);
            diag -= D[i][j];
        }
        D[i][i] = diag;
    }
    long double bp[kMaxPP], bm[kMaxPP];
    for (int side = 0; side < 2; ++side) {
        const long double t = side ? 1.0L : -1.0L;
        long double den = 0.0L;
        for (int k = 0; k < n; ++k) den += lam[k] / (t - x[k]);
        for (int j = 0; j < n; ++j) (side ? bp : bm)[j] = (lam[j] / (t - x[j])) / den;
    }
    for (int side = 0; side < 2; ++side) {
        const long double* b = side ? bp : bm;
        long double lp = 0.0L, lm = 0.0L;
        for (int m = 0; m < n; ++m) {
            lp += b[m] * bp[m] / w[m];
            lm += b[m] * bm[m] / w[m];
        }
        T.lface_p[side] = (double)lp;
        T.lface_m[side] = (double)lm;
        for (int l = 0; l < n; ++l) {
            long double acc = 0.0L;
            for (int m = 0; m < n; ++m) acc += b[m] * (D[l][m] * w[l] / w[m]);
            T.dface[side][l] = (double)acc;
        }
    }
    for (int i = 0; i < n; ++i) {
        T.nodes[i] = (double)x[i];
        T.w[i] = (double)w[i];
        T.bp[i] = (double)bp[i];
        T.bm[i] = (double)bm[i];
        T.bpw[i] = (double)(bp[i] / w[i]);
        T.bmw[i] = (double)(bm[i] / w[i]);
        for (int j = 0; j < n; ++j) {
            T.D[i * n + j] = (double)D[i][j];
            T.Dhat[i * n + j] = (double)(D[j][i] * w[j] / w[i]);
        }
    }
}

// 1D filter G1[a][j] from P_src to P_dst nodes (Sec. 2: nodal -> modal -> truncate -> nodal)
static void host_filter(int Ps, int Pd, double* G1) {
    BasisTab S, Dt;
    host_basis(Ps, S);
    host_basis(Pd, Dt);
    const int ns = Ps + 1, nd = Pd + 1;
    for (int a = 0; a < nd; ++a)
        for (int j = 0; j < ns; ++j) {
            long double acc = 0.0L;
            for (int k = 0; k <= Pd; ++k) {
                long double La, dLa, Lj, dLj;
                legendre_ld(k, Dt.nodes[a], La, dLa);
                legendre_ld(k, S.nodes[j], Lj, dLj);
                acc += La * (2 * k + 1) / 2.0L * (long double)S.w[j] * Lj;
            }
            G1[a * ns + j] = (double)acc;
        }
}

static std::mutex g_tab_mu;
static bool g_tab_done[kMaxDevices];

// once per device, with that device current: basis tables and the address
// of the no-alloc stepper's scratch
static int ensure_tables(int dev) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    if (dev < 0 || dev >= kMaxDevices) return set_error(DG_EINVAL, "device index %d out of range", dev);
    if (g_tab_done[dev]) return DG_OK;
    std::vector<BasisTab> tabs(DG_MAX_ORDER);
    for (int P = 1; P <= DG_MAX_ORDER; ++P) host_basis(P, tabs[P - 1]);
    DG_HIP(upload_basis_tables(tabs.data()));
    DG_HIP(scratch_setup(dev));
    g_tab_done[dev] = true;
    return DG_OK;
}

void fill_phys(const dg_params& p, Phys& ph) {
    std::memset(&ph, 0, sizeof(ph));
    ph.gamma = p.gamma;
    ph.gm1 = p.gamma - 1.0;
    ph.p_ref = p.p_ref;
    ph.mu = 1.0 / p.Re;
    ph.kappa = ph.mu * p.gamma / (ph.gm1 * p.Pr);
    ph.h = p.L / p.N;
    ph.L = p.L;
    ph.s = 2.0 / ph.h;
    ph.les = p.Cs > 0.0 ? 1 : 0;
    const double delta = ph.h / (p.P + 1);
    ph.les_c = ph.les ? (p.Cs * delta) * (p.Cs * delta) : 0.0;
    ph.kt = ph.les ? p.gamma / (ph.gm1 * p.Pr_t) : 0.0;
    ph.p0 = 1.0 / (p.gamma * p.Mach * p.Mach);
    ph.viscous = p.viscous ? 1 : 0;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout ws_layout(const Mesh& m) {
    WsLayout L;
    size_t off = 0;
    const size_t E = (size_t)m.E;
    L.desc = off;     off += align256(4 * sizeof(SolveDesc));
    L.qtr0 = off;     off += align256(E * 6 * 5 * m.n_f * sizeof(double));
    L.qtr1 = off;     off += align256(E * 6 * 5 * m.n_f * sizeof(double));
    L.fv = off;       off += align256(E * 6 * 4 * m.n_f * sizeof(double));
    L.forcing = off;  off += align256(E * 5 * m.n_p * sizeof(double));
    L.partial = off;  off += align256(E * 8 * sizeof(double) + 64 * sizeof(double));
    L.total = off;
    return L;
}

static SolveDesc make_desc(const Mesh& m, char* ws, const WsLayout& L) {
    SolveDesc d;
    std::memset(&d, 0, sizeof(d));
    d.N = m.N;
    d.E = m.E;
    d.ph = m.ph;
    d.fv = (double*)(ws + L.fv);
    return d;
}

static int check_mesh(const dg_mesh* m) {
    if (!m) return set_error(DG_EINVAL, "null mesh");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(DG_EHIP, "hipGetDevice failed");
    if (dev != m->m.device)
        return set_error(DG_EINVAL, "mesh was built on device %d, current device is %d", m->m.device, dev);
    return DG_OK;
}

static int check_ws(const Mesh& m, const void* ws, size_t ws_bytes) {
    if (!ws) return set_error(DG_EINVAL, "null workspace");
    if (((uintptr_t)ws) & 255) return set_error(DG_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = ws_layout(m).total;
    if (ws_bytes < need) return set_error(DG_ENOSPC, "workspace %zu bytes < %zu needed", ws_bytes, need);
    return DG_OK;
}

static bool aligned8(const void* p) { return (((uintptr_t)p) & 7) == 0; }

DescList single_list(const SolveDesc* d, int E) {
    DescList dl;
    std::memset(&dl, 0, sizeof(dl));
    dl.d[0] = d;
    dl.blk[0] = 0;
    dl.blk[1] = E;
    dl.n = 1;
    return dl;
}

DescList single_list(const SolveDesc* d, const SolveDesc& host, int E) {
    DescList dl = single_list(d, E);
    dl.inl = 1;
    dl.d0 = host;
    return dl;
}

// ----------------------------------------------------------------- internal API used by server/nn

int residual_impl(const Mesh& m, const double* q, double* dqdt, char* ws, hipStream_t st) {
    const WsLayout L = ws_layout(m);
    SolveDesc d = make_desc(m, ws, L);
    d.q = const_cast<double*>(q);
    d.out = dqdt;
    d.qtr_in = (const double*)(ws + L.qtr0);
    d.qtr_out = (double*)(ws + L.qtr0);
    SolveDesc* dd = (SolveDesc*)(ws + L.desc);
    DG_HIP(launch_write_descs(&d, 1, dd, st));
    const DescList dl = single_list(dd, d, m.E);
    DG_HIP(launch_traces(m.PP, dl, st));
    if (m.ph.viscous) DG_HIP(launch_grad(m.PP, dl, st));
    DG_HIP(launch_resid(m.PP, 0, dl, 0.0, 0.0, 1, st));
    return DG_OK;
}

const double kRkA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double kRkB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

int rk_impl(const Mesh& m, double* q, double* k, double dt, int n_steps, const nn_model* model, int post,
            char* ws, hipStream_t st) {
    const WsLayout L = ws_layout(m);
    const double* fbuf = model ? (const double*)(ws + L.forcing) : nullptr;
    // d[par]: the stages; d[2 + par]: the last stage of a post-corrected step
    SolveDesc d[4];
    for (int p = 0; p < 4; ++p) {
        const int par = p & 1;
        d[p] = make_desc(m, ws, L);
        d[p].q = q;
        d[p].k = k;
        d[p].dt = dt;
        d[p].forcing = post ? nullptr : fbuf;
        d[p].post = (post && p >= 2) ? fbuf : nullptr;
        d[p].qtr_in = (const double*)(ws + (par == 0 ? L.qtr0 : L.qtr1));
        d[p].qtr_out = (double*)(ws + (par == 0 ? L.qtr1 : L.qtr0));
    }
    SolveDesc* dd = (SolveDesc*)(ws + L.desc);
    DG_HIP(launch_write_descs(d, 4, dd, st));
    DescList dl[4];
    for (int p = 0; p < 4; ++p) dl[p] = single_list(dd + p, d[p], m.E);
    DG_HIP(launch_traces(m.PP, dl[1], st));   // traces of q into qtr0
    // P = 3 on a mesh that fills the GPU with 16-element blocks: the BR1
    // pass and the network in one launch, at every stage (Eq. (4)) or, for
    // the post-step correction (Algorithm 1), at the first stage, whose BR1
    // pass reads the same state q^n the network is evaluated on
    const bool fused = model && grad_net_fusable(model, m);
    int par = 0;
    for (int n = 0; n < n_steps; ++n) {
        // post-step correction (Algorithm 1): s from the state at the start of the step
        if (model && post && !fused) {
            int rc = net_forcing_impl(model, m, q, (double*)(ws + L.forcing), /*accumulate=*/0, st);
            if (rc != DG_OK) return rc;
        }
        for (int s = 0; s < 3; ++s) {
            const DescList& l = dl[(post && model && s == 2 ? 2 : 0) + par];
            if (fused && (!post || s == 0)) {
                int rc = grad_net_impl(model, m, l, q, (double*)(ws + L.forcing), st);
                if (rc != DG_OK) return rc;
            } else {
                if (m.ph.viscous) DG_HIP(launch_grad(m.PP, l, st));
                if (model && !post) {
                    int rc = net_forcing_impl(model, m, q, (double*)(ws + L.forcing), /*accumulate=*/0, st);
                    if (rc != DG_OK) return rc;
                }
            }
            DG_HIP(launch_resid(m.PP, 1, l, kRkA[s], kRkB[s], s == 0, st));
            par ^= 1;
        }
    }
    return DG_OK;
}

int diag_impl(const Mesh& m, const double* q, double* out_dev, char* ws, hipStream_t st) {
    const WsLayout L = ws_layout(m);
    DG_HIP(launch_diag(m.PP, m.ph, m.N, q, (double*)(ws + L.partial), out_dev, st));
    return DG_OK;
}

int project_impl(const Mesh& src, const Mesh& dst, const double* f_src, double* f_dst, hipStream_t st) {
    double G1[kMaxPP * kMaxPP];
    host_filter(src.P, dst.P, G1);
    DG_HIP(launch_project(src.PP, dst.PP, src.E, G1, f_src, f_dst, st));
    return DG_OK;
}

int init_tgv_impl(const Mesh& m, double* q, hipStream_t st) {
    DG_HIP(launch_tgv(m.PP, m.ph, m.N, q, st));
    return DG_OK;
}

double stable_dt_from_diag(const Mesh& m, const double* diag_host, double cfl) {
    const double n = m.PP;
    const double dt_a = cfl * m.ph.h / (n * n * diag_host[1]);
    const double nu = m.ph.mu / diag_host[2];
    const double diff = std::fmax(nu, m.prm.gamma * nu / m.prm.Pr);
    const double dt_v = cfl * m.ph.h * m.ph.h / (n * n * n * n * diff);
    return std::fmin(dt_a, dt_v);
}

int make_mesh(const dg_params* prm, Mesh& M) {
    if (!prm) return set_error(DG_EINVAL, "null params");
    const dg_params& p = *prm;
    if (p.P < DG_MIN_ORDER || p.P > DG_MAX_ORDER)
        return set_error(DG_EINVAL, "P = %d outside [%d, %d]", p.P, DG_MIN_ORDER, DG_MAX_ORDER);
    if (p.N < 1 || p.N > 1024) return set_error(DG_EINVAL, "N = %d outside [1, 1024]", p.N);
    const double n3 = (double)p.N * p.N * p.N;
    if (n3 * (p.P + 1) * (p.P + 1) * (p.P + 1) * 6.0 > 2.0e9)
        return set_error(DG_EINVAL, "mesh too large for 32-bit face indexing (N = %d, P = %d)", p.N, p.P);
    if (!(p.L > 0) || !(p.Re > 0) || !(p.Mach > 0) || !(p.gamma > 1) || !(p.Pr > 0) || !(p.Cs >= 0) ||
        (p.Cs > 0 && !(p.Pr_t > 0)) || !std::isfinite(p.p_ref))
        return set_error(DG_EINVAL, "invalid physical parameters");
    std::memset(&M, 0, sizeof(M));
    M.prm = p;
    M.N = p.N;
    M.P = p.P;
    M.PP = p.P + 1;
    M.E = p.N * p.N * p.N;
    M.n_p = M.PP * M.PP * M.PP;
    M.n_f = M.PP * M.PP;
    fill_phys(p, M.ph);
    int dev = 0;
    DG_HIP(hipGetDevice(&dev));
    M.device = dev;
    return ensure_tables(dev);
}

}  // namespace dgnn

using namespace dgnn;

extern "C" {

int dg_last_error(char* buf, size_t len) {
    if (!buf || len == 0) return DG_EINVAL;
    std::snprintf(buf, len, "%s", g_err.c_str());
    return DG_OK;
}

int dg_init_mesh(const dg_params* prm, dg_mesh** out) {
    if (!out) return set_error(DG_EINVAL, "null output handle");
    *out = nullptr;
    Mesh M;
    int rc = make_mesh(prm, M);
    if (rc != DG_OK) return rc;
    dg_mesh* m = new dg_mesh;
    m->m = M;
    *out = m;
    return DG_OK;
}

int dg_mesh_query(const dg_mesh* m, int64_t* n_nodes, size_t* workspace_bytes) {
    if (!m) return set_error(DG_EINVAL, "null mesh");
    if (n_nodes) *n_nodes = (int64_t)m->m.E * m->m.n_p;
    if (workspace_bytes) *workspace_bytes = ws_layout(m->m).total;
    return DG_OK;
}

void dg_free_mesh(dg_mesh* m) { delete m; }

int dg_init_tgv(const dg_mesh* m, double* q, void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !aligned8(q)) return set_error(DG_EINVAL, "bad state pointer");
    return init_tgv_impl(m->m, q, (hipStream_t)stream);
}

int dg_residual(const dg_mesh* m, const double* q, double* dqdt, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !dqdt || !aligned8(q) || !aligned8(dqdt)) return set_error(DG_EINVAL, "bad state pointers");
    if (q == dqdt) return set_error(DG_EINVAL, "q and dqdt alias");
    if ((rc = check_ws(m->m, ws, ws_bytes))) return rc;
    return residual_impl(m->m, q, dqdt, (char*)ws, (hipStream_t)stream);
}

int dg_rk_step(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps, const nn_model* forcing,
               void* ws, size_t ws_bytes, void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !k || !aligned8(q) || !aligned8(k)) return set_error(DG_EINVAL, "bad state pointers");
    if (q == k) return set_error(DG_EINVAL, "q and k alias");
    if (!(dt > 0) || !std::isfinite(dt)) return set_error(DG_EINVAL, "dt must be positive and finite");
    if (n_steps < 0) return set_error(DG_EINVAL, "negative step count");
    if ((rc = check_ws(m->m, ws, ws_bytes))) return rc;
    if (forcing && (rc = net_check_mesh(forcing, m->m))) return rc;
    if (n_steps == 0) return DG_OK;
    return rk_impl(m->m, q, k, dt, n_steps, forcing, 0, (char*)ws, (hipStream_t)stream);
}

int dg_rk_step_post(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps, const nn_model* forcing,
                    void* ws, size_t ws_bytes, void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !k || !aligned8(q) || !aligned8(k)) return set_error(DG_EINVAL, "bad state pointers");
    if (q == k) return set_error(DG_EINVAL, "q and k alias");
    if (!(dt > 0) || !std::isfinite(dt)) return set_error(DG_EINVAL, "dt must be positive and finite");
    if (n_steps < 0) return set_error(DG_EINVAL, "negative step count");
    if ((rc = check_ws(m->m, ws, ws_bytes))) return rc;
    if (forcing && (rc = net_check_mesh(forcing, m->m))) return rc;
    if (n_steps == 0) return DG_OK;
    return rk_impl(m->m, q, k, dt, n_steps, forcing, 1, (char*)ws, (hipStream_t)stream);
}

int dg_rk_step_noalloc(const dg_mesh* m, double* q, double* k, double dt, int32_t n_steps, const nn_model* forcing,
                       void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !k || !aligned8(q) || !aligned8(k)) return set_error(DG_EINVAL, "bad state pointers");
    if (q == k) return set_error(DG_EINVAL, "q and k alias");
    if (!(dt > 0) || !std::isfinite(dt)) return set_error(DG_EINVAL, "dt must be positive and finite");
    if (n_steps < 0) return set_error(DG_EINVAL, "negative step count");
    const size_t need = ws_layout(m->m).total;
    if (need > DG_NOALLOC_SCRATCH_BYTES)
        return set_error(DG_ENOSPC, "N = %d, P = %d needs %zu bytes of workspace; the no-alloc scratch holds %zu",
                         m->m.N, m->m.P, need, (size_t)DG_NOALLOC_SCRATCH_BYTES);
    char* ws = (char*)scratch_device_ptr(m->m.device);
    if (!ws) return set_error(DG_EHIP, "no-alloc scratch not set up on device %d", m->m.device);
    if (forcing && (rc = net_check_mesh(forcing, m->m))) return rc;
    if (n_steps == 0) return DG_OK;
    return rk_impl(m->m, q, k, dt, n_steps, forcing, 0, ws, (hipStream_t)stream);
}

int dg_profile_steps(const dg_mesh* mh, double* q, double* k, double dt, int32_t n_steps, const nn_model* model,
                     void* ws_v, size_t ws_bytes, void* stream, double* out_ms) {
    int rc = check_mesh(mh);
    if (rc) return rc;
    if (!q || !k || q == k || !out_ms) return set_error(DG_EINVAL, "bad pointers");
    if (!(dt > 0) || n_steps < 1) return set_error(DG_EINVAL, "dt must be positive and n_steps >= 1");
    if ((rc = check_ws(mh->m, ws_v, ws_bytes))) return rc;
    if (model && (rc = net_check_mesh(model, mh->m))) return rc;
    const Mesh& m = mh->m;
    char* ws = (char*)ws_v;
    hipStream_t st = (hipStream_t)stream;
    const WsLayout L = ws_layout(m);
    SolveDesc d[2];
    for (int p = 0; p < 2; ++p) {
        d[p] = make_desc(m, ws, L);
        d[p].q = q;
        d[p].k = k;
        d[p].dt = dt;
        d[p].forcing = model ? (const double*)(ws + L.forcing) : nullptr;
        d[p].qtr_in = (const double*)(ws + (p == 0 ? L.qtr0 : L.qtr1));
        d[p].qtr_out = (double*)(ws + (p == 0 ? L.qtr1 : L.qtr0));
    }
    SolveDesc* dd = (SolveDesc*)(ws + L.desc);
    DG_HIP(launch_write_descs(d, 2, dd, st));
    const DescList dl[2] = {single_list(dd, d[0], m.E), single_list(dd + 1, d[1], m.E)};
    const int n_ev = 2 * (1 + 9 * n_steps);
    std::vector<hipEvent_t> ev(n_ev);
    for (auto& e : ev) DG_HIP(hipEventCreate(&e));
    std::vector<int> kind;
    int ie = 0;
    auto mark = [&](int kd) -> hipError_t {
        kind.push_back(kd);
        return hipEventRecord(ev[ie++], st);
    };
    int err = DG_OK;
    do {
        if (mark(0) != hipSuccess || launch_traces(m.PP, dl[1], st) != hipSuccess || hipEventRecord(ev[ie++], st) != hipSuccess) {
            err = set_error(DG_EHIP, "trace launch failed");
            break;
        }
        const bool fused = model && grad_net_fusable(model, m);
        int par = 0;
        for (int n = 0; n < n_steps && err == DG_OK; ++n)
            for (int s = 0; s < 3 && err == DG_OK; ++s) {
                if (fused) {
                    // the fused BR1-and-network launch, timed as the network's
                    if (mark(2) != hipSuccess) err = set_error(DG_EHIP, "event failed");
                    else if ((err = grad_net_impl(model, m, dl[par], q, (double*)(ws + L.forcing), st)) == DG_OK &&
                             hipEventRecord(ev[ie++], st) != hipSuccess)
                        err = set_error(DG_EHIP, "event failed");
                } else if (m.ph.viscous) {
                    if (mark(1) != hipSuccess || launch_grad(m.PP, dl[par], st) != hipSuccess ||
                        hipEventRecord(ev[ie++], st) != hipSuccess)
                        err = set_error(DG_EHIP, "grad launch failed");
                }
                if (model && !fused && err == DG_OK) {
                    if (mark(2) != hipSuccess) err = set_error(DG_EHIP, "event failed");
                    else if ((err = net_forcing_impl(model, m, q, (double*)(ws + L.forcing), 0, st)) == DG_OK &&
                             hipEventRecord(ev[ie++], st) != hipSuccess)
                        err = set_error(DG_EHIP, "event failed");
                }
                if (err == DG_OK && (mark(3) != hipSuccess ||
                                     launch_resid(m.PP, 1, dl[par], kRkA[s], kRkB[s], s == 0, st) != hipSuccess ||
                                     hipEventRecord(ev[ie++], st) != hipSuccess))
                    err = set_error(DG_EHIP, "resid launch failed");
                par ^= 1;
            }
    } while (0);
    if (err == DG_OK && hipStreamSynchronize(st) != hipSuccess) err = set_error(DG_EHIP, "synchronise failed");
    double sum[4] = {0, 0, 0, 0};
    int cnt[4] = {0, 0, 0, 0};
    if (err == DG_OK)
        for (size_t i = 0; i < kind.size(); ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) {
                err = set_error(DG_EHIP, "event timing failed");
                break;
            }
            sum[kind[i]] += ms;
            cnt[kind[i]] += 1;
        }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (err) return err;
    for (int c = 0; c < 4; ++c) out_ms[c] = cnt[c] ? sum[c] / cnt[c] : 0.0;
    return DG_OK;
}

int dg_diagnostics(const dg_mesh* m, const double* q, double* out_dev, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !out_dev) return set_error(DG_EINVAL, "null pointer");
    if ((rc = check_ws(m->m, ws, ws_bytes))) return rc;
    return diag_impl(m->m, q, out_dev, (char*)ws, (hipStream_t)stream);
}

int dg_stable_dt(const dg_mesh* m, const double* q, double cfl, double* dt_host, void* ws, size_t ws_bytes,
                 void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !dt_host) return set_error(DG_EINVAL, "null pointer");
    if (!(cfl > 0)) return set_error(DG_EINVAL, "cfl must be positive");
    if ((rc = check_ws(m->m, ws, ws_bytes))) return rc;
    const WsLayout L = ws_layout(m->m);
    double* out = (double*)((char*)ws + L.partial) + (size_t)m->m.E * 8;   // 64 spare doubles
    hipStream_t st = (hipStream_t)stream;
    if ((rc = diag_impl(m->m, q, out, (char*)ws, st))) return rc;
    double h[8];
    DG_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(h[1]) || !(h[2] > 0)) return set_error(DG_ENONFINITE, "state is not finite/positive");
    *dt_host = stable_dt_from_diag(m->m, h, cfl);
    return DG_OK;
}

int dg_error_inf(const dg_mesh* m, const double* q, const double* q_ref, double* out_dev, void* ws,
                 size_t ws_bytes, void* stream) {
    int rc = check_mesh(m);
    if (rc) return rc;
    if (!q || !q_ref || !out_dev) return set_error(DG_EINVAL, "null pointer");
    if ((rc = check_ws(m->m, ws, ws_bytes))) return rc;
    const WsLayout L = ws_layout(m->m);
    DG_HIP(launch_err_inf(m->m.PP, m->m.E, q, q_ref, (double*)((char*)ws + L.partial), out_dev,
                          (hipStream_t)stream));
    return DG_OK;
}

int dg_project(const dg_mesh* src, const dg_mesh* dst, const double* f_src, double* f_dst, void* stream) {
    int rc = check_mesh(src);
    if (rc) return rc;
    if ((rc = check_mesh(dst))) return rc;
    if (src->m.N != dst->m.N) return set_error(DG_EINVAL, "meshes differ in N");
    if (dst->m.P > src->m.P) return set_error(DG_EINVAL, "destination order above source order");
    if (!f_src || !f_dst || f_src == f_dst) return set_error(DG_EINVAL, "bad field pointers");
    return project_impl(src->m, dst->m, f_src, f_dst, (hipStream_t)stream);
}

size_t dg_forcing_target_ws(const dg_mesh* hi, const dg_mesh* lo) {
    if (!hi || !lo) return 0;
    const size_t E = hi->m.E;
    size_t b = 0;
    b += align256(E * 5 * hi->m.n_p * sizeof(double));   // R_hi
    b += 3 * align256(E * 5 * lo->m.n_p * sizeof(double)); // Gq, GR, R_lo
    b += ws_layout(hi->m).total;                           // residual workspaces (reused)
    b += ws_layout(lo->m).total;
    return b;
}

int dg_forcing_target(const dg_mesh* hi, const dg_mesh* lo, const double* q_hi, float* x_out, float* y_out,
                      void* ws, size_t ws_bytes, void* stream) {
    int rc = check_mesh(hi);
    if (rc) return rc;
    if ((rc = check_mesh(lo))) return rc;
    if (hi->m.N != lo->m.N || lo->m.P > hi->m.P) return set_error(DG_EINVAL, "incompatible meshes");
    if (!q_hi || !x_out || !y_out) return set_error(DG_EINVAL, "null pointer");
    if (!ws || (((uintptr_t)ws) & 255)) return set_error(DG_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = dg_forcing_target_ws(hi, lo);
    if (ws_bytes < need) return set_error(DG_ENOSPC, "workspace %zu bytes < %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    const size_t E = hi->m.E;
    char* p = (char*)ws;
    double* R_hi = (double*)p;  p += align256(E * 5 * hi->m.n_p * sizeof(double));
    double* Gq = (double*)p;    p += align256(E * 5 * lo->m.n_p * sizeof(double));
    double* GR = (double*)p;    p += align256(E * 5 * lo->m.n_p * sizeof(double));
    double* R_lo = (double*)p;  p += align256(E * 5 * lo->m.n_p * sizeof(double));
    char* ws_hi = p;            p += ws_layout(hi->m).total;
    char* ws_lo = p;
    if ((rc = residual_impl(hi->m, q_hi, R_hi, ws_hi, st))) return rc;
    if ((rc = project_impl(hi->m, lo->m, q_hi, Gq, st))) return rc;
    if ((rc = project_impl(hi->m, lo->m, R_hi, GR, st))) return rc;
    if ((rc = residual_impl(lo->m, Gq, R_lo, ws_lo, st))) return rc;
    DG_HIP(launch_pack_pairs(lo->m.E, lo->m.n_p, 1.0, Gq, GR, R_lo, x_out, y_out, st));
    return DG_OK;
}

}  // extern "C"

extern "C" {

size_t dg_increment_target_ws(const dg_mesh* hi, const dg_mesh* lo) {
    if (!hi || !lo) return 0;
    const size_t E = lo->m.E;
    return 4 * align256(E * 5 * lo->m.n_p * sizeof(double)) + ws_layout(hi->m).total + ws_layout(lo->m).total;
}

int dg_increment_target(const dg_mesh* hi, const dg_mesh* lo, double* q_hi, double* k_hi, double dt_lo,
                        int32_t m_sub, float* x_out, float* y_out, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_mesh(hi);
    if (rc) return rc;
    if ((rc = check_mesh(lo))) return rc;
    if (hi->m.N != lo->m.N || lo->m.P > hi->m.P) return set_error(DG_EINVAL, "incompatible meshes");
    if (!q_hi || !k_hi || q_hi == k_hi || !aligned8(q_hi) || !aligned8(k_hi) || !x_out || !y_out)
        return set_error(DG_EINVAL, "bad pointers");
    if (!(dt_lo > 0) || !std::isfinite(dt_lo)) return set_error(DG_EINVAL, "dt must be positive and finite");
    if (m_sub < 1) return set_error(DG_EINVAL, "m_sub must be >= 1");
    if (!ws || (((uintptr_t)ws) & 255)) return set_error(DG_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = dg_increment_target_ws(hi, lo);
    if (ws_bytes < need) return set_error(DG_ENOSPC, "workspace %zu bytes < %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    const size_t fb = align256((size_t)lo->m.E * 5 * lo->m.n_p * sizeof(double));
    char* p = (char*)ws;
    double* q_nn = (double*)p;   p += fb;   // q_NN^n = G q_HO^n
    double* q_nn1 = (double*)p;  p += fb;   // its uncorrected low-order step
    double* k_lo = (double*)p;   p += fb;
    double* qbar = (double*)p;   p += fb;   // G q_HO^{n+1}
    char* ws_hi = p;             p += ws_layout(hi->m).total;
    char* ws_lo = p;
    if ((rc = project_impl(hi->m, lo->m, q_hi, q_nn, st))) return rc;
    if ((rc = project_impl(hi->m, lo->m, q_hi, q_nn1, st))) return rc;
    if ((rc = rk_impl(lo->m, q_nn1, k_lo, dt_lo, 1, nullptr, 0, ws_lo, st))) return rc;
    if ((rc = rk_impl(hi->m, q_hi, k_hi, dt_lo / m_sub, m_sub, nullptr, 0, ws_hi, st))) return rc;
    if ((rc = project_impl(hi->m, lo->m, q_hi, qbar, st))) return rc;
    DG_HIP(launch_pack_pairs(lo->m.E, lo->m.n_p, dt_lo, q_nn, qbar, q_nn1, x_out, y_out, st));
    return DG_OK;
}

}  // extern "C"
