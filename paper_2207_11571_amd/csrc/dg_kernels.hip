// FP64 DGSEM kernels for gfx950: face traces, BR1 gradient pass, residual and
// Runge-Kutta stage update, Taylor-Green initial condition, diagnostics,
// filter G and training-pair packing.
//
// Discretisation (Sec. 2.6, Sec. 3.1, App. A): weak-form nodal DGSEM on
// Gauss-Legendre points, Roe interface flux, BR1 gradients of (u, v, w, T)
// and viscous fluxes, optional Smagorinsky closure, on uniform periodic
// hexahedra.  One workgroup owns one element; thread t owns node t
// (n = i + PP (j + PP k)); the element's state is staged in LDS so that the
// (P+1)-long line contractions of the sum-factorised operators read LDS.
//
// Per Runge-Kutta stage two kernels run (BR1 needs neighbours' gradients,
// which need their neighbours' traces):
//   k_grad  : q, neighbour q traces -> BR1 gradient (at P = 8 only its
//             face values) -> one-sided viscous normal flux on the element's
//             six faces (fv);
//   k_resid : q, neighbour q traces, fv of both sides -> Roe minus averaged
//             viscous interface flux, volume flux divergence, forcing ->
//             residual, or the low-storage stage update of q and k plus the
//             face traces of the new q for the next stage.
#include <mutex>

#include "dgnn_internal.hpp"
#include "nn_device.hpp"

namespace dgnn {

__constant__ BasisTab c_basis[DG_MAX_ORDER];

template <int PP>
struct Shape {
    static constexpr int NP = PP * PP * PP;
    static constexpr int NF = PP * PP;
    static constexpr int NT = ((NP + 63) / 64) * 64;
    static constexpr int NFT = 6 * NF;                  // face-node tasks
    static constexpr int TPT = (NFT + NT - 1) / NT;     // tasks per thread
    // minimum wavefronts per SIMD that the stage kernels are compiled for:
    // five lets three blocks of 4 - 6 wavefronts share a CU (P = 4 - 6;
    // P = 3 is bound by LDS, P >= 7 by the registers it needs), where the
    // kernel fits the registers that leaves without spilling; the residual
    // at P = 5 (x and y fluxes at once) needs more and runs four
    static constexpr int WPE = (PP == 5 || PP == 7) ? 5 : (PP == 6 ? 4 : 2);
    static constexpr int GRAD_WPE = (PP >= 5 && PP <= 7) ? 5 : 2;
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// The arrays a solve descriptor points to are addressed through gmem()
// (global memory): read from a descriptor in memory they are generic
// pointers, and generic (flat) accesses count against the LDS counter as
// well, so every LDS access would wait for the element's global loads and
// stores in flight.
using gdouble = global_t<double>;

__device__ __forceinline__ int find_solve(const DescList& dl, int b) {
    int s = 0;
    for (int i = 1; i < dl.n; ++i)
        if (dl.blk[i] <= b) s = i;
    return s;
}

// The neighbour across face f of element e at coordinates (cx, cy, cz)
// (uniform across the block), without an integer division per thread.
__device__ __forceinline__ int neighbour_at(int e, int N, int cx, int cy, int cz, int f) {
    const int d = f >> 1;
    const int cd = d == 0 ? cx : (d == 1 ? cy : cz);
    const int stride = d == 0 ? 1 : (d == 1 ? N : N * N);
    const int up = (cd + 1 == N) ? 1 - N : 1;
    const int down = (cd == 0) ? N - 1 : -1;
    return e + ((f & 1) ? up : down) * stride;
}

// node of the line through face-node (a, b) of a face normal to d, at position m
template <int PP>
__device__ __forceinline__ int line_node(int d, int a, int b, int m) {
    return d == 0 ? m + PP * (a + PP * b) : (d == 1 ? a + PP * (m + PP * b) : a + PP * (b + PP * m));
}

// --------------------------------------------------------------- physics

// 1/x for x > 0 normal: hardware estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r), each doubling the correct bits
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(x) for x > 0 normal: hardware 1/sqrt estimate y, then Goldschmidt's
// coupled iteration on g ~ sqrt(x), h ~ 1/(2 sqrt(x)) and a final residual
// correction g + h (x - g^2)
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

// value of the axis-d entry of a triple, for a runtime axis
__device__ __forceinline__ double pick3(int d, double x0, double x1, double x2) {
    return d == 0 ? x0 : (d == 1 ? x1 : x2);
}

// w = (u, v, w, T) with T = p / rho
__device__ __forceinline__ void gradient_vars(const double q[5], double gm1, double w[4]) {
    const double ir = recip(q[0]);
    w[0] = q[1] * ir;
    w[1] = q[2] * ir;
    w[2] = q[3] * ir;
    const double p = gm1 * (q[4] - 0.5 * (q[1] * w[0] + q[2] * w[1] + q[3] * w[2]));
    w[3] = p * ir;
}

// Roe flux along +D, qL on the lower side (Roe 1981), no entropy fix
template <int D>
__device__ void flux_roe(const double qL[5], const double qR[5], const Phys& ph, double F[5]) {
    const double gm1 = ph.gm1;
    const double rL = qL[0], rR = qR[0];
    const double iL = recip(rL), iR = recip(rR);
    double vL[3], vR[3];
    for (int a = 0; a < 3; ++a) { vL[a] = qL[1 + a] * iL; vR[a] = qR[1 + a] * iR; }
    const double pL = gm1 * (qL[4] - 0.5 * rL * (vL[0] * vL[0] + vL[1] * vL[1] + vL[2] * vL[2]));
    const double pR = gm1 * (qR[4] - 0.5 * rR * (vR[0] * vR[0] + vR[1] * vR[1] + vR[2] * vR[2]));
    const double HL = (qL[4] + pL) * iL, HR = (qR[4] + pR) * iR;
    const double sL = sqrt_pos(rL), sR = sqrt_pos(rR);
    const double rt = sL * sR;
    const double isum = recip(sL + sR);
    double vt[3];
    for (int a = 0; a < 3; ++a) vt[a] = (sL * vL[a] + sR * vR[a]) * isum;
    const double Ht = (sL * HL + sR * HR) * isum;
    const double v2 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
    const double ct = sqrt_pos(gm1 * (Ht - 0.5 * v2));
    const double vn = vt[D];
    const double ic2 = recip(ct * ct);
    const double dr = rR - rL, dp = pR - pL;
    double dv[3];
    for (int a = 0; a < 3; ++a) dv[a] = vR[a] - vL[a];
    // wave strengths times |eigenvalue|
    const double wm = fabs(vn - ct) * (dp - rt * ct * dv[D]) * 0.5 * ic2;
    const double wp = fabs(vn + ct) * (dp + rt * ct * dv[D]) * 0.5 * ic2;
    const double l0 = fabs(vn);
    const double we = l0 * (dr - dp * ic2);
    double diss[5];
    diss[0] = wm + we + wp;
    double de = wm * (Ht - ct * vn) + we * 0.5 * v2 + wp * (Ht + ct * vn);
    for (int a = 0; a < 3; ++a) {
        double m = (wm + we + wp) * vt[a];
        if (a == D) {
            m += (wp - wm) * ct;
        } else {
            const double ws = l0 * rt * dv[a];   // shear wave
            m += ws;
            de += ws * vt[a];
        }
        diss[1 + a] = m;
    }
    diss[4] = de;
    double FL[5], FR[5];
    // central part from the primitive values already at hand
    {
        const double vdL = vL[D], vdR = vR[D];
        FL[0] = qL[1 + D];  FR[0] = qR[1 + D];
        FL[1] = qL[1] * vdL; FR[1] = qR[1] * vdR;
        FL[2] = qL[2] * vdL; FR[2] = qR[2] * vdR;
        FL[3] = qL[3] * vdL; FR[3] = qR[3] * vdR;
        FL[1 + D] += pL - ph.p_ref;
        FR[1 + D] += pR - ph.p_ref;
        FL[4] = (qL[4] + pL) * vdL;
        FR[4] = (qR[4] + pR) * vdR;
    }
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * diss[v];
}

// Effective viscosity and conductivity: mu, kappa plus, with the Smagorinsky
// closure, mu_t = rho (Cs Delta)^2 sqrt(2 S:S) and mu_t gamma/((gamma-1) Pr_t).
__device__ __forceinline__ void effective_visc(double rho, const double g[3][4], const Phys& ph, double& mu,
                                               double& kappa) {
    mu = ph.mu;
    kappa = ph.kappa;
    if (ph.les) {
        double SS = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double Sab = 0.5 * (g[a][b] + g[b][a]);
                SS += Sab * Sab;
            }
        const double mut = rho * ph.les_c * sqrt(2.0 * SS);
        mu += mut;
        kappa += mut * ph.kt;
    }
}

// One-sided viscous flux along D (App. A): momentum rows tau_{aD} and the
// energy row sum_a v_a tau_{aD} + kappa dT/dx_D.  g[j][c] = d_j w_c.
template <int D>
__device__ __forceinline__ void flux_viscous(double rho, const double v[3], const double g[3][4],
                                             const Phys& ph, double Fv[4]) {
    double mu, kappa;
    effective_visc(rho, g, ph, mu, kappa);
    const double div = g[0][0] + g[1][1] + g[2][2];
    double e = 0.0;
    for (int a = 0; a < 3; ++a) {
        double tau = mu * (g[a][D] + g[D][a]);
        if (a == D) tau -= (2.0 / 3.0) * mu * div;
        Fv[a] = tau;
        e += v[a] * tau;
    }
    Fv[3] = e + kappa * g[D][3];
}

// Node quantities that the three directions of the volume flux share:
// velocity, p - p_ref (momentum rows), rho E + p (energy row) and, viscous,
// the symmetric stress tau (tau_00, tau_11, tau_22, tau_01, tau_02, tau_12,
// with the Smagorinsky viscosity when on) and the energy rows
// sum_a v_a tau_aD + kappa dT/dx_D of the three directions.  The gradient is
// dead after this, which keeps the register budget of the volume phase low.
struct NodeState {
    double v[3], pt, pe, tau[6], ev[3];
};

__device__ __forceinline__ int sym_index(int a, int b) {
    return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

__device__ __forceinline__ void node_state(const double q[5], const double g[3][4], const Phys& ph, NodeState& n) {
    const double ir = recip(q[0]);
    n.v[0] = q[1] * ir;
    n.v[1] = q[2] * ir;
    n.v[2] = q[3] * ir;
    const double p = ph.gm1 * (q[4] - 0.5 * (q[1] * n.v[0] + q[2] * n.v[1] + q[3] * n.v[2]));
    n.pt = p - ph.p_ref;
    n.pe = q[4] + p;
    if (ph.viscous) {
        double mu, kappa;
        effective_visc(q[0], g, ph, mu, kappa);
        const double lam = (2.0 / 3.0) * mu * (g[0][0] + g[1][1] + g[2][2]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                double t = mu * (g[a][b] + g[b][a]);
                if (a == b) t -= lam;
                n.tau[sym_index(a, b)] = t;
            }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double e = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) e += n.v[a] * n.tau[sym_index(a, d)];
            n.ev[d] = e + kappa * g[d][3];
        }
    }
}

// net volume flux along D: inviscid (App. A, p_ref removed from the momentum
// rows) minus viscous
template <int D>
__device__ __forceinline__ void flux_net(const double q[5], const NodeState& n, const Phys& ph, double G[5]) {
    const double vd = n.v[D];
    G[0] = q[1 + D];
    G[1] = q[1] * vd;
    G[2] = q[2] * vd;
    G[3] = q[3] * vd;
    G[1 + D] += n.pt;
    G[4] = n.pe * vd;
    if (ph.viscous) {
#pragma unroll
        for (int a = 0; a < 3; ++a) G[1 + a] -= n.tau[sym_index(a, D)];
        G[4] -= n.ev[D];
    }
}

// One-sided viscous flux across a face normal to axis d: flux_viscous<0> of
// the velocity and gradient with axes relabelled cyclically so that d comes
// first (both the derivative axis and the velocity component), relabelled
// back; one code path for the three orientations.
__device__ __forceinline__ void flux_viscous_rot(int d, double rho, const double v[3], const double g[3][4],
                                                 const Phys& ph, double Fv[4]) {
    // entry (r, c) of the relabelled gradient is entry ((r + d) mod 3, (c + d) mod 3)
    double vr[3], gr[3][4];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        vr[r] = pick3(d, v[r], v[(r + 1) % 3], v[(r + 2) % 3]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            gr[r][c] = pick3(d, g[r][c], g[(r + 1) % 3][(c + 1) % 3], g[(r + 2) % 3][(c + 2) % 3]);
        gr[r][3] = pick3(d, g[r][3], g[(r + 1) % 3][3], g[(r + 2) % 3][3]);
    }
    double Fr[4];
    flux_viscous<0>(rho, vr, gr, ph, Fr);
    Fv[0] = pick3(d, Fr[0], Fr[2], Fr[1]);
    Fv[1] = pick3(d, Fr[1], Fr[0], Fr[2]);
    Fv[2] = pick3(d, Fr[2], Fr[1], Fr[0]);
    Fv[3] = Fr[3];
}

// Roe flux across a face normal to axis d (qL on the lower side): the
// x-direction flux of the states with their axes relabelled cyclically so
// that d comes first (rotated momentum r is original momentum (r + d) mod 3),
// relabelled back.  One code path serves the three orientations, so the
// lanes of a wavefront whose face nodes straddle faces of different
// orientation run the flux once instead of once per orientation under masks.
__device__ __forceinline__ void flux_roe_rot(int d, const double qL[5], const double qR[5], const Phys& ph,
                                             double F[5]) {
    double a[5], b[5];
    a[0] = qL[0];
    b[0] = qR[0];
    a[4] = qL[4];
    b[4] = qR[4];
    a[1] = pick3(d, qL[1], qL[2], qL[3]);
    a[2] = pick3(d, qL[2], qL[3], qL[1]);
    a[3] = pick3(d, qL[3], qL[1], qL[2]);
    b[1] = pick3(d, qR[1], qR[2], qR[3]);
    b[2] = pick3(d, qR[2], qR[3], qR[1]);
    b[3] = pick3(d, qR[3], qR[1], qR[2]);
    double G[5];
    flux_roe<0>(a, b, ph, G);
    F[0] = G[0];
    F[4] = G[4];
    F[1] = pick3(d, G[1], G[3], G[2]);
    F[2] = pick3(d, G[2], G[1], G[3]);
    F[3] = pick3(d, G[3], G[2], G[1]);
}

// ----------------------------------------------------- element-local pieces

// trace of the nodal field sh[v*NP + n] (v < nv) on face f at face node fn
template <int PP, int NV>
__device__ __forceinline__ void face_interp(const double* __restrict__ sh, const BasisTab& B, int f, int fn,
                                            double out[NV]) {
    constexpr int NP = PP * PP * PP;
    const int d = f >> 1;
    const int a = fn % PP, b = fn / PP;
    const double* bv = (f & 1) ? B.bp : B.bm;
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    if constexpr (NV <= 5) {
#pragma unroll
        for (int m = 0; m < PP; ++m) {
            const int n = line_node<PP>(d, a, b, m);
            const double c = bv[m];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] += c * sh[v * NP + n];
        }
    } else {
        // wide interpolations (the 12 gradient components): a partial unroll
        // keeps the loads in flight within the register budget of large blocks
#pragma unroll 3
        for (int m = 0; m < PP; ++m) {
            const int n = line_node<PP>(d, a, b, m);
            const double c = bv[m];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] += c * sh[v * NP + n];
        }
    }
}

// weak-form derivative along D at node t of the nodal field sh[c*NP + .] with
// interface values fhat[(f*NC + c)*NF + fn]:
//   s [ b+_i/w_i Fhat(+) - b-_i/w_i Fhat(-) - sum_m Dhat[i][m] F_m ]
template <int PP, int D, int NC>
__device__ __forceinline__ void weak_deriv(const double* __restrict__ sh, const double* __restrict__ fhat,
                                           const BasisTab& B, int t, double s, double out[NC]) {
    constexpr int NP = PP * PP * PP;
    constexpr int NF = PP * PP;
    constexpr int stride = D == 0 ? 1 : (D == 1 ? PP : PP * PP);
    const int i = t % PP, j = (t / PP) % PP, k = t / (PP * PP);
    const int id = D == 0 ? i : (D == 1 ? j : k);
    const int fn = D == 0 ? j + PP * k : (D == 1 ? i + PP * k : i + PP * j);
    const int base = t - id * stride;
    double acc[NC];
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
#pragma unroll
    for (int m = 0; m < PP; ++m) {
        const double dm = B.Dhat[id * PP + m];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += dm * sh[c * NP + base + m * stride];
    }
    const double lp = B.bpw[id], lm = B.bmw[id];
    const int fp = 2 * D + 1, fm = 2 * D;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        out[c] = s * (lp * fhat[(fp * NC + c) * NF + fn] - lm * fhat[(fm * NC + c) * NF + fn] - acc[c]);
}

template <int PP>
struct Lines {
    static constexpr int NF = PP * PP;
    static constexpr int NLT = 3 * NF;                             // line tasks
    static constexpr int LPT = (NLT + Shape<PP>::NT - 1) / Shape<PP>::NT;   // tasks per thread
};

// traces of the nodal field sh[v*NP + n] (v < NV) at both ends of a line
template <int PP, int NV>
__device__ __forceinline__ void line_interp(const double* __restrict__ sh, const BasisTab& B, int d, int fn,
                                            double om[NV], double op[NV]) {
    constexpr int NP = PP * PP * PP;
    const int a = fn % PP, b = fn / PP;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        om[v] = 0.0;
        op[v] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < PP; ++m) {
        const int n = line_node<PP>(d, a, b, m);
        const double cm = B.bm[m], cp = B.bp[m];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double x = sh[v * NP + n];
            om[v] += cm * x;
            op[v] += cp * x;
        }
    }
}

// the six face traces of the nodal state in LDS, to global
template <int PP>
__device__ __forceinline__ void write_traces(const double* __restrict__ sh, const BasisTab& B, int t, int e,
                                             gdouble* __restrict__ out) {
    using S = Shape<PP>;
    using Ln = Lines<PP>;
#pragma unroll
    for (int r = 0; r < Ln::LPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < Ln::NLT) {
            const int d = tau / S::NF, fn = tau - d * S::NF;
            double qm[5], qp[5];
            line_interp<PP, 5>(sh, B, d, fn, qm, qp);
            gdouble* om = out + (size_t)(e * 6 + 2 * d) * 5 * S::NF + fn;
            gdouble* op = om + 5 * S::NF;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                om[v * S::NF] = qm[v];
                op[v * S::NF] = qp[v];
            }
        }
    }
}

// ---------------------------------------------------------------- kernels

template <int PP>
__global__ void __launch_bounds__(Shape<PP>::NT) k_traces(DescList dl) {
    using S = Shape<PP>;
    __shared__ double sh[5 * S::NP];
    const int b = blockIdx.x;
    const int si = find_solve(dl, b);
    const SolveDesc& D = *dl.d[si];
    const int e = b - dl.blk[si];
    const int E = D.E;
    const int t = threadIdx.x;
    const BasisTab& B = c_basis[PP - 2];
    if (t < S::NP)
        for (int v = 0; v < 5; ++v) sh[v * S::NP + t] = gmem(D.q)[((size_t)v * E + e) * S::NP + t];
    __syncthreads();
    write_traces<PP>(sh, B, t, e, gmem(D.qtr_out));
}

// BR1 pass, volume form: the lifted gradient at every node, then its face
// interpolation.
template <int PP>
struct GradLds {
    static constexpr int N = cmax(12 * Shape<PP>::NP, 5 * Shape<PP>::NP + 24 * Shape<PP>::NF);
};

// The barrier between two phases of one element's work: the block's, or,
// where one wavefront owns the element and its LDS area, that wavefront's
// (its LDS operations complete in order, so the fences only keep the
// compiler from moving LDS accesses across it).
template <bool WAVE>
__device__ __forceinline__ void element_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// element e of solve D, thread t of the element's Shape<PP>::NT, LDS area sh
// of GradLds<PP>::N doubles; the node's state is left in qn (t < NP).  WAVE:
// the element is one wavefront's alone (Shape<PP>::NT == 64)
template <int PP, bool WAVE = false>
__device__ __forceinline__ void grad_volume_element(const SolveDesc& D, int e, int t, double* __restrict__ sh,
                                                    double qn[5]) {
    using S = Shape<PP>;
    static_assert(!WAVE || S::NT == 64, "a wavefront per element");
    constexpr int NP = S::NP, NF = S::NF;
    double* what = sh + 5 * NP;                  // [6][4][NF] common BR1 values
    const Phys ph = D.ph;
    const int ecx = e % D.N, ecy = (e / D.N) % D.N, ecz = e / (D.N * D.N);
    const int E = D.E;
    const BasisTab& B = c_basis[PP - 2];

    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qn[v] = gmem(D.q)[((size_t)v * E + e) * NP + t];
    }

    double fq[S::TPT][4];   // own traced (rho, u, v, w) per face task
#pragma unroll
    for (int r = 0; r < S::TPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < S::NFT) {
            const int f = tau / NF, fn = tau - f * NF;
            double qi[5], qo[5];
            // the element's own trace on this face, written with the state
            // by the trace epilogue (the same line interpolation of the
            // same values, so the same numbers as interpolating sh here)
            const gdouble* ti = gmem(D.qtr_in) + (size_t)(e * 6 + f) * 5 * NF + fn;
#pragma unroll
            for (int v = 0; v < 5; ++v) qi[v] = ti[v * NF];
            const int nb = neighbour_at(e, D.N, ecx, ecy, ecz, f);
            const gdouble* tr = gmem(D.qtr_in) + (size_t)(nb * 6 + (f ^ 1)) * 5 * NF + fn;
#pragma unroll
            for (int v = 0; v < 5; ++v) qo[v] = tr[v * NF];
            double wi[4], wo[4];
            gradient_vars(qi, ph.gm1, wi);
            gradient_vars(qo, ph.gm1, wo);
#pragma unroll
            for (int c = 0; c < 4; ++c) what[(f * 4 + c) * NF + fn] = 0.5 * (wi[c] + wo[c]);
            fq[r][0] = qi[0];
            fq[r][1] = wi[0];
            fq[r][2] = wi[1];
            fq[r][3] = wi[2];
        }
    }
    if (t < NP) {
        double w[4];
        gradient_vars(qn, ph.gm1, w);
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[c * NP + t] = w[c];
    }
    element_sync<WAVE>();
    double g[3][4];
    if (t < NP) {
        weak_deriv<PP, 0, 4>(sh, what, B, t, ph.s, g[0]);
        weak_deriv<PP, 1, 4>(sh, what, B, t, ph.s, g[1]);
        weak_deriv<PP, 2, 4>(sh, what, B, t, ph.s, g[2]);
    }
    element_sync<WAVE>();
    if (t < NP) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 4; ++c) sh[(d * 4 + c) * NP + t] = g[d][c];
    }
    element_sync<WAVE>();
#pragma unroll
    for (int r = 0; r < S::TPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < S::NFT) {
            const int f = tau / NF, fn = tau - f * NF;
            double gi[12];
            face_interp<PP, 12>(sh, B, f, fn, gi);
            double gf[3][4];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int c = 0; c < 4; ++c) gf[d][c] = gi[d * 4 + c];
            const double v[3] = {fq[r][1], fq[r][2], fq[r][3]};
            double Fv[4];
            flux_viscous_rot(f >> 1, fq[r][0], v, gf, ph, Fv);
            gdouble* o = gmem(D.fv) + (size_t)(e * 6 + f) * 4 * NF + fn;
#pragma unroll
            for (int c = 0; c < 4; ++c) o[c * NF] = Fv[c];
        }
    }
}

template <int PP>
__device__ __forceinline__ void grad_volume_form(const DescList& dl) {
    __shared__ double sh[GradLds<PP>::N];
    const int b = blockIdx.x;
    const int si = find_solve(dl, b);
    double qn[5];
    grad_volume_element<PP>(*dl.d[si], b - dl.blk[si], threadIdx.x, sh, qn);
}

// BR1 pass, face form: only the face values of the lifted gradient are needed here, so they are
// formed on the faces directly (sum factorisation): the normal derivative as
// one line contraction with the end-evaluated derivative row, the two
// tangential derivatives as contractions of the face trace of w along the
// face, with the lifting terms of the tangential faces interpolated to the
// face's edges.  The result equals the face interpolation of the volume
// gradient up to rounding, at O(P^3) instead of O(P^4) work per element.
template <int PP>
struct GradFaceLds {
    static constexpr int NET = 24 * PP;          // edge tasks: 6 faces x 2 tangential axes x 2 sides x PP
    static constexpr int N = 5 * Shape<PP>::NP + 48 * Shape<PP>::NF + 4 * NET;
};

// element e of solve D, thread t, basis B, LDS area sh of GradFaceLds<PP>::N
template <int PP>
__device__ __forceinline__ void grad_face_element(const SolveDesc& D, int e, int t, const BasisTab& B,
                                                  double* __restrict__ sh) {
    using S = Shape<PP>;
    constexpr int NP = S::NP, NF = S::NF;
    constexpr int NET = GradFaceLds<PP>::NET;
    double* what = sh + 5 * NP;                  // [6][4][NF] common BR1 values
    double* wf = what + 24 * NF;                 // [6][4][NF] face traces of w
    double* edge = wf + 24 * NF;                 // [6][2][2][4][PP] lifting values at the face edges
    const Phys ph = D.ph;
    const int ecx = e % D.N, ecy = (e / D.N) % D.N, ecz = e / (D.N * D.N);
    const int E = D.E;

    double qn[5];
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qn[v] = gmem(D.q)[((size_t)v * E + e) * NP + t];
    }

    double fq[S::TPT][4];   // own traced (rho, u, v, w) per face task
#pragma unroll
    for (int r = 0; r < S::TPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < S::NFT) {
            const int f = tau / NF, fn = tau - f * NF;
            double qi[5], qo[5];
            // the element's own trace on this face, written with the state
            // by the trace epilogue (the same line interpolation of the
            // same values, so the same numbers as interpolating sh here)
            const gdouble* ti = gmem(D.qtr_in) + (size_t)(e * 6 + f) * 5 * NF + fn;
#pragma unroll
            for (int v = 0; v < 5; ++v) qi[v] = ti[v * NF];
            const int nb = neighbour_at(e, D.N, ecx, ecy, ecz, f);
            const gdouble* tr = gmem(D.qtr_in) + (size_t)(nb * 6 + (f ^ 1)) * 5 * NF + fn;
#pragma unroll
            for (int v = 0; v < 5; ++v) qo[v] = tr[v * NF];
            double wi[4], wo[4];
            gradient_vars(qi, ph.gm1, wi);
            gradient_vars(qo, ph.gm1, wo);
#pragma unroll
            for (int c = 0; c < 4; ++c) what[(f * 4 + c) * NF + fn] = 0.5 * (wi[c] + wo[c]);
            fq[r][0] = qi[0];
            fq[r][1] = wi[0];
            fq[r][2] = wi[1];
            fq[r][3] = wi[2];
        }
    }
    if (t < NP) {
        double w[4];
        gradient_vars(qn, ph.gm1, w);
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[c * NP + t] = w[c];
    }
    __syncthreads();
    // edge values: the common values of a tangential face pair (axis dp,
    // side sg), interpolated along the face normal to the face's edge
    for (int tau = t; tau < NET; tau += S::NT) {
        const int r = tau % PP, rest = tau / PP;
        const int sg = rest & 1, u = (rest >> 1) & 1, f = rest >> 2;
        const int d = f >> 1;
        const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        const int dp = u ? t1 : t0, dpp = u ? t0 : t1;
        const double* bv = (f & 1) ? B.bp : B.bm;
        const double* src = what + (2 * dp + sg) * 4 * NF;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < PP; ++m) {
            const int fnp = d < dpp ? m + PP * r : r + PP * m;
            const double c0 = bv[m];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += c0 * src[c * NF + fnp];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) edge[(rest * 4 + c) * PP + r] = acc[c];
    }
    // the face traces of w: independent of the edge values (both read only
    // what the first barrier published), so no barrier between them
#pragma unroll
    for (int r = 0; r < S::TPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < S::NFT) {
            const int f = tau / NF, fn = tau - f * NF;
            double wv[4];
            face_interp<PP, 4>(sh, B, f, fn, wv);
#pragma unroll
            for (int c = 0; c < 4; ++c) wf[(f * 4 + c) * NF + fn] = wv[c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < S::TPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < S::NFT) {
            const int f = tau / NF, fn = tau - f * NF;
            const int d = f >> 1, sd = f & 1;
            const int a = fn % PP, bb = fn / PP;
            // normal derivative: the line's weak derivative at this end
            double gn[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int l = 0; l < PP; ++l) {
                const double c0 = B.dface[sd][l];
                const int n = line_node<PP>(d, a, bb, l);
#pragma unroll
                for (int c = 0; c < 4; ++c) gn[c] += c0 * sh[c * NP + n];
            }
            const double lp = B.lface_p[sd], lm = B.lface_m[sd];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                gn[c] = ph.s * (lp * what[((2 * d + 1) * 4 + c) * NF + fn] - lm * what[(2 * d * 4 + c) * NF + fn] - gn[c]);
            // tangential derivatives along the face's first (a) and second (b) axis
            double ga[4] = {0.0, 0.0, 0.0, 0.0}, gb[4] = {0.0, 0.0, 0.0, 0.0};
            const double* wfp = wf + f * 4 * NF;
#pragma unroll
            for (int l = 0; l < PP; ++l) {
                const double ca = B.Dhat[a * PP + l], cb = B.Dhat[bb * PP + l];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    ga[c] += ca * wfp[c * NF + l + PP * bb];
                    gb[c] += cb * wfp[c * NF + a + PP * l];
                }
            }
            const double* ef = edge + f * 16 * PP;       // [u][side][c][PP]
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ga[c] = ph.s * (B.bpw[a] * ef[(4 + c) * PP + bb] - B.bmw[a] * ef[c * PP + bb] - ga[c]);
                gb[c] = ph.s * (B.bpw[bb] * ef[(12 + c) * PP + a] - B.bmw[bb] * ef[(8 + c) * PP + a] - gb[c]);
            }
            // back to the element's axes: the normal is d, the face's first
            // axis the lower of the other two
            double gf[3][4];
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const bool first = (x == 0 && d != 0) || (x == 1 && d == 0);
                    gf[x][c] = x == d ? gn[c] : (first ? ga[c] : gb[c]);
                }
            const double v[3] = {fq[r][1], fq[r][2], fq[r][3]};
            double Fv[4];
            flux_viscous_rot(d, fq[r][0], v, gf, ph, Fv);
            gdouble* o = gmem(D.fv) + (size_t)(e * 6 + f) * 4 * NF + fn;
#pragma unroll
            for (int c = 0; c < 4; ++c) o[c * NF] = Fv[c];
        }
    }
}

// BR1 pass: one-sided viscous normal fluxes on the six faces of each
// element.  The face form does less arithmetic but more index work per face
// node; measured, it is the faster one at P = 8 only.
template <int PP>
__device__ __forceinline__ void grad_face_form(const DescList& dl) {
    __shared__ double sh[GradFaceLds<PP>::N];
    const int b = blockIdx.x;
    const int si = find_solve(dl, b);
    grad_face_element<PP>(*dl.d[si], b - dl.blk[si], threadIdx.x, c_basis[PP - 2], sh);
}

template <int PP>
__global__ void __launch_bounds__(Shape<PP>::NT) __attribute__((amdgpu_waves_per_eu(Shape<PP>::GRAD_WPE)))
k_grad(DescList dl) {
    if constexpr (PP >= 9) grad_face_form<PP>(dl);
    else grad_volume_form<PP>(dl);
}

// the same for one solve whose descriptor is in the kernel arguments
template <int PP>
__global__ void __launch_bounds__(Shape<PP>::NT) __attribute__((amdgpu_waves_per_eu(Shape<PP>::GRAD_WPE)))
k_grad1(DescList dl) {
    if constexpr (PP >= 9) {
        __shared__ double sh[GradFaceLds<PP>::N];
        grad_face_element<PP>(dl.d0, blockIdx.x, threadIdx.x, c_basis[PP - 2], sh);
    } else {
        __shared__ double sh[GradLds<PP>::N];
        double qn[5];
        grad_volume_element<PP>(dl.d0, blockIdx.x, threadIdx.x, sh, qn);
    }
}

// P = 3 with the forcing network at every stage (Eq. (4)): the BR1 pass of
// sixteen elements, one per wavefront, and the network on the same sixteen
// rows in one launch.  Each wavefront works on its own element in its own
// LDS area, so between the BR1 pass's phases it waits for itself only, not
// for the block.  After the BR1 pass each wavefront holds its
// element's state in registers (node n in lane n), so it writes the
// element's normalised network input row straight into LDS instead of the
// network gathering the state from HBM again, and the layers follow in the
// same block.  The same device code as k_grad and k_net_forcing, so the same
// numbers.  One solve per launch (its descriptor in the kernel arguments),
// E a multiple of 16.
template <int PP>
__global__ void __launch_bounds__(kRowThreads) k_grad_net(DescList dl, NetArgs na, NetTarget T) {
    using S = Shape<PP>;
    static_assert(S::NT == 64 && S::NP == 64, "one element per wavefront, one node per lane");
    constexpr int NP = S::NP;
    extern __shared__ __attribute__((aligned(16))) double gsm[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int pmax = 0;
    for (int l = 0; l <= na.n_layers; ++l) pmax = pmax > na.pdims[l] ? pmax : na.pdims[l];
    const int ld = pmax + kLdPad;
    uint16_t* bufA = (uint16_t*)(gsm + kRowWaves * GradLds<PP>::N);
    uint16_t* bufB = bufA + kRows * ld;
    const SolveDesc& D = dl.d0;   // one solve, its descriptor in the arguments
    const int e0 = blockIdx.x * kRows;

    double qn[5];
    grad_volume_element<PP, true>(D, e0 + wave, lane, gsm + wave * GradLds<PP>::N, qn);

    // row `wave` of the network input: column j NP + n is node n of
    // variable in_var[j]
    const int din = na.dims[0], pin = na.pdims[0];
    uint16_t* row = bufA + wave * ld;
    for (int j = 0; j < na.n_in; ++j) {
        const int v = na.in_var[j];
        const double qv = v == 0 ? qn[0] : (v == 1 ? qn[1] : (v == 2 ? qn[2] : (v == 3 ? qn[3] : qn[4])));
        row[j * NP + lane] = f2bf(net_input(na, NP, v, lane, qv));
    }
    for (int c = din + lane; c < pin; c += 64) row[c] = f2bf(0.0f);
    net_zero_unforced(na, NP, T, e0, threadIdx.x);
    __syncthreads();
    net_block_forward(na, NP, T, e0, 0, bufA, bufB, ld, wave, lane);
}

template <int PP>
struct ResidLds {
    // P = 8 (one block per CU): the three directions' node fluxes are
    // stored at once, so the flux divergence needs one barrier, not six
    static constexpr bool DIV3 = PP >= 9;
    // P = 5, 6: the x and y node fluxes at once (four barriers instead of
    // six; the LDS still lets three blocks share a CU)
    static constexpr bool DIV2 = PP >= 6 && PP <= 7;
    static constexpr int N = (DIV3 ? 20 : (DIV2 ? 10 : 5)) * Shape<PP>::NP + 54 * Shape<PP>::NF;
};

// element e of solve D, thread t of the element's Shape<PP>::NT, basis B,
// LDS area sh of ResidLds<PP>::N doubles
template <int PP, int UPDATE>
__device__ __forceinline__ void resid_element(const SolveDesc& D, int e, int t, const BasisTab& B,
                                              double* __restrict__ sh, double rkA, double rkB, int first_stage) {
    using S = Shape<PP>;
    constexpr int NP = S::NP, NF = S::NF;
    constexpr bool DIV3 = ResidLds<PP>::DIV3;
    constexpr bool DIV2 = ResidLds<PP>::DIV2;
    double* fhat = sh + (DIV3 ? 20 : (DIV2 ? 10 : 5)) * NP;   // [6][5][NF] net interface flux
    double* G3 = sh + 5 * NP;                     // DIV3: [3][5][NP] node fluxes
    double* what = fhat + 30 * NF;       // [6][4][NF] common BR1 values
    const Phys ph = D.ph;
    const int ecx = e % D.N, ecy = (e / D.N) % D.N, ecz = e / (D.N * D.N);
    const int E = D.E;
    const size_t node = (size_t)e * NP + t;
    const size_t vstride = (size_t)E * NP;

    // The face phase works on traces only, so the node's own state goes
    // straight to registers: loaded with the face data, and the Runge-Kutta
    // register with it, where registers are to spare (P = 8, one block per
    // CU), otherwise after the face phase.
    constexpr bool QEARLY = PP >= 9;
    double qn[5], kp[5];
    if (QEARLY && t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qn[v] = gmem(D.q)[v * vstride + node];
        if (UPDATE && !first_stage) {
#pragma unroll
            for (int v = 0; v < 5; ++v) kp[v] = gmem(D.k)[v * vstride + node];
        }
        // the gradient variables go to LDS with the face phase's values,
        // behind the same barrier
        if (ph.viscous) {
            double w[4];
            gradient_vars(qn, ph.gm1, w);
#pragma unroll
            for (int c = 0; c < 4; ++c) sh[c * NP + t] = w[c];
        }
    }

#pragma unroll
    for (int r = 0; r < S::TPT; ++r) {
        const int tau = t + r * S::NT;
        if (tau < S::NFT) {
            const int f = tau / NF, fn = tau - f * NF;
            const int d = f >> 1;
            double qi[5], qo[5];
            // the element's own trace on this face, written with the state
            // by the trace epilogue (the same line interpolation of the
            // same values, so the same numbers as interpolating sh here)
            const gdouble* ti = gmem(D.qtr_in) + (size_t)(e * 6 + f) * 5 * NF + fn;
#pragma unroll
            for (int v = 0; v < 5; ++v) qi[v] = ti[v * NF];
            const int nb = neighbour_at(e, D.N, ecx, ecy, ecz, f);
            const gdouble* tr = gmem(D.qtr_in) + (size_t)(nb * 6 + (f ^ 1)) * 5 * NF + fn;
#pragma unroll
            for (int v = 0; v < 5; ++v) qo[v] = tr[v * NF];
            // the lower-side state is the neighbour's on a lower face
            const bool up = f & 1;
            double qL[5], qR[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qL[v] = up ? qi[v] : qo[v];
                qR[v] = up ? qo[v] : qi[v];
            }
            double F[5];
            flux_roe_rot(d, qL, qR, ph, F);
            if (ph.viscous) {
                const gdouble* fi = gmem(D.fv) + (size_t)(e * 6 + f) * 4 * NF + fn;
                const gdouble* fo = gmem(D.fv) + (size_t)(nb * 6 + (f ^ 1)) * 4 * NF + fn;
#pragma unroll
                for (int c = 0; c < 4; ++c) F[1 + c] -= 0.5 * (fi[c * NF] + fo[c * NF]);
                double wi[4], wo[4];
                gradient_vars(qi, ph.gm1, wi);
                gradient_vars(qo, ph.gm1, wo);
#pragma unroll
                for (int c = 0; c < 4; ++c) what[(f * 4 + c) * NF + fn] = 0.5 * (wi[c] + wo[c]);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) fhat[(f * 5 + v) * NF + fn] = F[v];
        }
    }
    __syncthreads();

    if (!QEARLY && t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qn[v] = gmem(D.q)[v * vstride + node];
    }
    double g[3][4];
    if (ph.viscous) {
        if (!QEARLY) {
            if (t < NP) {
                double w[4];
                gradient_vars(qn, ph.gm1, w);
#pragma unroll
                for (int c = 0; c < 4; ++c) sh[c * NP + t] = w[c];
            }
            __syncthreads();
        }
        if (t < NP) {
            weak_deriv<PP, 0, 4>(sh, what, B, t, ph.s, g[0]);
            weak_deriv<PP, 1, 4>(sh, what, B, t, ph.s, g[1]);
            weak_deriv<PP, 2, 4>(sh, what, B, t, ph.s, g[2]);
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 4; ++c) g[d][c] = 0.0;
    }

    NodeState ns;
    if (t < NP) node_state(qn, g, ph, ns);
    double R[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (DIV3) {
        if (t < NP) {
            double G[5];
            flux_net<0>(qn, ns, ph, G);
#pragma unroll
            for (int v = 0; v < 5; ++v) G3[v * NP + t] = G[v];
            flux_net<1>(qn, ns, ph, G);
#pragma unroll
            for (int v = 0; v < 5; ++v) G3[(5 + v) * NP + t] = G[v];
            flux_net<2>(qn, ns, ph, G);
#pragma unroll
            for (int v = 0; v < 5; ++v) G3[(10 + v) * NP + t] = G[v];
        }
        __syncthreads();
        if (t < NP) {
            double dv[5];
            weak_deriv<PP, 0, 5>(G3, fhat, B, t, ph.s, dv);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] -= dv[v];
            weak_deriv<PP, 1, 5>(G3 + 5 * NP, fhat, B, t, ph.s, dv);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] -= dv[v];
            weak_deriv<PP, 2, 5>(G3 + 10 * NP, fhat, B, t, ph.s, dv);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] -= dv[v];
        }
    } else if constexpr (DIV2) {
        __syncthreads();
        if (t < NP) {
            double G[5];
            flux_net<0>(qn, ns, ph, G);
#pragma unroll
            for (int v = 0; v < 5; ++v) sh[v * NP + t] = G[v];
            flux_net<1>(qn, ns, ph, G);
#pragma unroll
            for (int v = 0; v < 5; ++v) sh[(5 + v) * NP + t] = G[v];
        }
        __syncthreads();
        if (t < NP) {
            double dv[5];
            weak_deriv<PP, 0, 5>(sh, fhat, B, t, ph.s, dv);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] -= dv[v];
            weak_deriv<PP, 1, 5>(sh + 5 * NP, fhat, B, t, ph.s, dv);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] -= dv[v];
        }
        __syncthreads();
        if (t < NP) {
            double G[5];
            flux_net<2>(qn, ns, ph, G);
#pragma unroll
            for (int v = 0; v < 5; ++v) sh[v * NP + t] = G[v];
        }
        __syncthreads();
        if (t < NP) {
            double dv[5];
            weak_deriv<PP, 2, 5>(sh, fhat, B, t, ph.s, dv);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[v] -= dv[v];
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            __syncthreads();
            if (t < NP) {
                double G[5];
                if (d == 0) flux_net<0>(qn, ns, ph, G);
                else if (d == 1) flux_net<1>(qn, ns, ph, G);
                else flux_net<2>(qn, ns, ph, G);
#pragma unroll
                for (int v = 0; v < 5; ++v) sh[v * NP + t] = G[v];
            }
            __syncthreads();
            if (t < NP) {
                double dv[5];
                if (d == 0) weak_deriv<PP, 0, 5>(sh, fhat, B, t, ph.s, dv);
                else if (d == 1) weak_deriv<PP, 1, 5>(sh, fhat, B, t, ph.s, dv);
                else weak_deriv<PP, 2, 5>(sh, fhat, B, t, ph.s, dv);
#pragma unroll
                for (int v = 0; v < 5; ++v) R[v] -= dv[v];
            }
        }
    }

    if (t < NP && D.forcing) {
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] += gmem(D.forcing)[v * vstride + node];
    }

    if (!UPDATE) {
        if (t < NP) {
#pragma unroll
            for (int v = 0; v < 5; ++v) gmem(D.out)[v * vstride + node] = R[v];
        }
        return;
    }

    // the trace buffer's address read before the update's stores (after
    // them the compiler would read it from the descriptor again)
    gdouble* const qtr_out = gmem(D.qtr_out);
    if (t < NP) {
        // every load of the update (the Runge-Kutta register, the post-step
        // correction) issued before the first store, and the descriptor's
        // fields read once: after a store the compiler reloads them, and a
        // load after each store would cost a round trip per variable
        const double dt = D.dt;
        gdouble* kg = gmem(D.k);
        gdouble* qg = gmem(D.q);
        const double* postp = D.post;
        double kold[5], pst[5];
        if (!first_stage) {
#pragma unroll
            for (int v = 0; v < 5; ++v) kold[v] = QEARLY ? kp[v] : kg[v * vstride + node];
        }
        if (postp) {
#pragma unroll
            for (int v = 0; v < 5; ++v) pst[v] = gmem(postp)[v * vstride + node];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double kk = first_stage ? dt * R[v] : rkA * kold[v] + dt * R[v];
            qn[v] += rkB * kk;
            if (postp) qn[v] += dt * pst[v];
            kg[v * vstride + node] = kk;
            qg[v * vstride + node] = qn[v];
        }
    }
    // the new state goes to an LDS area no thread reads any more: the first
    // five fields (DIV3: its node fluxes live above them), the x-y flux
    // fields (DIV2: read before the z fluxes were written), else after a
    // barrier
    double* qs = DIV2 ? sh + 5 * NP : sh;
    if (!DIV3 && !DIV2) __syncthreads();
    if (t < NP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qs[v * NP + t] = qn[v];
    }
    __syncthreads();
    write_traces<PP>(qs, B, t, e, qtr_out);
}

// Residual (update == 0: out = p(q) + forcing) or Runge-Kutta stage
// (update == 1: k <- A k + dt R, q <- q + B k, traces of the new q), one
// element per block.
template <int PP, int UPDATE>
__global__ void __launch_bounds__(Shape<PP>::NT) __attribute__((amdgpu_waves_per_eu(Shape<PP>::WPE)))
k_resid(DescList dl, double rkA, double rkB, int first_stage) {
    __shared__ double sh[ResidLds<PP>::N];
    const int b = blockIdx.x;
    const int si = find_solve(dl, b);
    resid_element<PP, UPDATE>(*dl.d[si], b - dl.blk[si], threadIdx.x, c_basis[PP - 2], sh, rkA, rkB, first_stage);
}

// the same for one solve whose descriptor is in the kernel arguments
template <int PP, int UPDATE>
__global__ void __launch_bounds__(Shape<PP>::NT) __attribute__((amdgpu_waves_per_eu(Shape<PP>::WPE)))
k_resid1(DescList dl, double rkA, double rkB, int first_stage) {
    __shared__ double sh[ResidLds<PP>::N];
    resid_element<PP, UPDATE>(dl.d0, blockIdx.x, threadIdx.x, c_basis[PP - 2], sh, rkA, rkB, first_stage);
}

// The same for one solve whose blocks fill a CU each (P = 8): one block per
// CU walks the elements b, b + G, b + 2G, ... (G blocks), which spares the
// launch of a block per element and lets each block's next element start as
// soon as it is done with the last.  The descriptor is read once, at entry
// (inside the loop, after the loop's own stores, the compiler could only
// read it with vector loads that wait for those stores).
template <int PP, int UPDATE>
__global__ void __launch_bounds__(Shape<PP>::NT) __attribute__((amdgpu_waves_per_eu(Shape<PP>::WPE)))
k_resid_loop(DescList dl, double rkA, double rkB, int first_stage) {
    __shared__ double sh[ResidLds<PP>::N];
    const SolveDesc D = *dl.d[0];
    for (int e = blockIdx.x; e < D.E; e += gridDim.x) {
        // the thread index and the basis table made opaque per element, so
        // that what derives from them (line and face indices, basis entries)
        // is recomputed instead of being held in registers across the loop
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        int bz = 0;
        asm volatile("" : "+s"(bz));
        resid_element<PP, UPDATE>(D, e, t, c_basis[PP - 2 + bz], sh, rkA, rkB, first_stage);
        __syncthreads();
    }
}

// Taylor-Green vortex initial condition, Eq. (11), on [0, L]^3.
template <int PP>
__global__ void __launch_bounds__(Shape<PP>::NT) k_tgv(Phys ph, int N, double* __restrict__ q) {
    using S = Shape<PP>;
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    if (t >= S::NP) return;
    const BasisTab& B = c_basis[PP - 2];
    const int i = t % PP, j = (t / PP) % PP, k = t / (PP * PP);
    const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
    const double h = ph.h;
    const double x = ex * h + (B.nodes[i] + 1.0) * h * 0.5;
    const double y = ey * h + (B.nodes[j] + 1.0) * h * 0.5;
    const double z = ez * h + (B.nodes[k] + 1.0) * h * 0.5;
    const double u = sin(x) * cos(y) * cos(z);
    const double v = -cos(x) * sin(y) * cos(z);
    const double p = ph.p0 + (cos(2.0 * x) + cos(2.0 * y)) * (cos(2.0 * z) + 2.0) / 16.0;
    const size_t vs = (size_t)N * N * N * S::NP;
    const size_t n = (size_t)e * S::NP + t;
    q[n] = 1.0;
    q[vs + n] = u;
    q[2 * vs + n] = v;
    q[3 * vs + n] = 0.0;
    q[4 * vs + n] = p / ph.gm1 + 0.5 * (u * u + v * v);
}

// Per-element partial diagnostics: KE integrand sum, max(|v| + c), min rho,
// integrals of the five conserved variables (quadrature-weighted).  Fixed
// reduction order, so the result is bitwise reproducible.
template <int PP>
__global__ void __launch_bounds__(256) k_diag_partial(Phys ph, int E, const double* __restrict__ q,
                                                     double* __restrict__ part) {
    constexpr int NP = PP * PP * PP;
    __shared__ double red[8][256];
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    const BasisTab& B = c_basis[PP - 2];
    double val[8] = {0.0, 0.0, 1e300, 0.0, 0.0, 0.0, 0.0, 0.0};
    const size_t vs = (size_t)E * NP;
    for (int n = t; n < NP; n += 256) {
        const int i = n % PP, j = (n / PP) % PP, k = n / (PP * PP);
        const double wq = B.w[i] * B.w[j] * B.w[k];
        double qq[5];
        for (int v = 0; v < 5; ++v) qq[v] = q[v * vs + (size_t)e * NP + n];
        const double ir = 1.0 / qq[0];
        const double m2 = qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3];
        val[0] += wq * 0.5 * m2 * ir;
        const double p = ph.gm1 * (qq[4] - 0.5 * m2 * ir);
        val[1] = fmax(val[1], sqrt(m2) * ir + sqrt(ph.gamma * p * ir));
        val[2] = fmin(val[2], qq[0]);
        for (int v = 0; v < 5; ++v) val[3 + v] += wq * qq[v];
    }
    for (int c = 0; c < 8; ++c) red[c][t] = val[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] = fmax(red[1][t], red[1][t + w]);
            red[2][t] = fmin(red[2][t], red[2][t + w]);
            for (int c = 3; c < 8; ++c) red[c][t] += red[c][t + w];
        }
        __syncthreads();
    }
    if (t < 8) part[(size_t)e * 8 + t] = red[t][0];
}

__global__ void __launch_bounds__(256) k_diag_final(int E, double vol_factor, const double* __restrict__ part,
                                                   double* __restrict__ out) {
    __shared__ double red[8][256];
    const int t = threadIdx.x;
    double val[8] = {0.0, 0.0, 1e300, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = t; e < E; e += 256) {
        const double* p = part + (size_t)e * 8;
        val[0] += p[0];
        val[1] = fmax(val[1], p[1]);
        val[2] = fmin(val[2], p[2]);
        for (int c = 3; c < 8; ++c) val[c] += p[c];
    }
    for (int c = 0; c < 8; ++c) red[c][t] = val[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] = fmax(red[1][t], red[1][t + w]);
            red[2][t] = fmin(red[2][t], red[2][t + w]);
            for (int c = 3; c < 8; ++c) red[c][t] += red[c][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        // vol_factor = J: integrals; KE is the volume mean, J / L^3 folded in by the caller
        out[0] = red[0][0];
        out[1] = red[1][0];
        out[2] = red[2][0];
        for (int c = 3; c < 8; ++c) out[c] = red[c][0] * vol_factor;
    }
}

__global__ void k_scale(double* p, double f) {
    if (threadIdx.x == 0) p[0] *= f;
}

// Eq. (9): per-element max |q_v - qref_v| for the three momenta
__global__ void __launch_bounds__(256) k_err_partial(int E, int NP, const double* __restrict__ q,
                                                    const double* __restrict__ qr, double* __restrict__ part) {
    __shared__ double red[3][256];
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    double m[3] = {0.0, 0.0, 0.0};
    const size_t vs = (size_t)E * NP;
    for (int n = t; n < NP; n += 256)
        for (int c = 0; c < 3; ++c) {
            const size_t idx = (1 + c) * vs + (size_t)e * NP + n;
            m[c] = fmax(m[c], fabs(q[idx] - qr[idx]));
        }
    for (int c = 0; c < 3; ++c) red[c][t] = m[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 3; ++c) red[c][t] = fmax(red[c][t], red[c][t + w]);
        __syncthreads();
    }
    if (t < 3) part[(size_t)e * 3 + t] = red[t][0];
}

__global__ void __launch_bounds__(256) k_err_final(int E, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    double m[3] = {0.0, 0.0, 0.0};
    for (int e = t; e < E; e += 256)
        for (int c = 0; c < 3; ++c) m[c] = fmax(m[c], part[(size_t)e * 3 + c]);
    for (int c = 0; c < 3; ++c) red[c][t] = m[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 3; ++c) red[c][t] = fmax(red[c][t], red[c][t + w]);
        __syncthreads();
    }
    if (t < 3) out[t] = red[t][0];
}

// Filter G: tensor-product 1D projection, one element per block, five variables.
struct ProjArg {
    double G[kMaxPP * kMaxPP];   // [PPd][PPs]
};

template <int PPS, int PPD>
__global__ void __launch_bounds__(256) k_project(ProjArg pa, int E, const double* __restrict__ src,
                                                double* __restrict__ dst) {
    constexpr int NS = PPS * PPS * PPS;
    constexpr int ND = PPD * PPD * PPD;
    __shared__ double G[PPD * PPS];
    __shared__ double a[5 * NS];
    __shared__ double b1[5 * PPD * PPS * PPS];
    __shared__ double b2[5 * PPD * PPD * PPS];
    const int e = blockIdx.x;
    const int t = threadIdx.x;
    for (int x = t; x < PPD * PPS; x += 256) G[x] = pa.G[x];
    const size_t vss = (size_t)E * NS, vsd = (size_t)E * ND;
    for (int x = t; x < 5 * NS; x += 256) {
        const int v = x / NS, n = x - v * NS;
        a[x] = src[v * vss + (size_t)e * NS + n];
    }
    __syncthreads();
    // along x: b1[v][k][j][i'] = sum_i G[i'][i] a[v][k][j][i]
    for (int x = t; x < 5 * PPS * PPS * PPD; x += 256) {
        const int ip = x % PPD, r = x / PPD;        // r = (v, k, j)
        double acc = 0.0;
        for (int i = 0; i < PPS; ++i) acc += G[ip * PPS + i] * a[r * PPS + i];
        b1[x] = acc;
    }
    __syncthreads();
    // along y: b2[v][k][j'][i'] = sum_j G[j'][j] b1[v][k][j][i']
    for (int x = t; x < 5 * PPS * PPD * PPD; x += 256) {
        const int ip = x % PPD, jp = (x / PPD) % PPD, r = x / (PPD * PPD);   // r = (v, k)
        double acc = 0.0;
        for (int j = 0; j < PPS; ++j) acc += G[jp * PPS + j] * b1[(r * PPS + j) * PPD + ip];
        b2[x] = acc;
    }
    __syncthreads();
    // along z
    for (int x = t; x < 5 * ND; x += 256) {
        const int ip = x % PPD, jp = (x / PPD) % PPD, kp = (x / (PPD * PPD)) % PPD, v = x / ND;
        double acc = 0.0;
        for (int k = 0; k < PPS; ++k) acc += G[kp * PPS + k] * b2[((v * PPS + k) * PPD + jp) * PPD + ip];
        dst[v * vsd + (size_t)e * ND + (x - v * ND)] = acc;
    }
}

__global__ void __launch_bounds__(256) k_pack_pairs(int E, int NP, double div, const double* __restrict__ Gq,
                                                   const double* __restrict__ GR, const double* __restrict__ R3,
                                                   float* __restrict__ x, float* __restrict__ y) {
    const size_t total = (size_t)5 * E * NP;
    const size_t vs = (size_t)E * NP;
    for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
        const int v = (int)(idx / vs);
        const size_t rem = idx - v * vs;
        const size_t e = rem / NP, n = rem - e * NP;
        const size_t o = e * (5 * NP) + (size_t)v * NP + n;
        x[o] = (float)Gq[idx];
        y[o] = (float)((GR[idx] - R3[idx]) / div);
    }
}

struct DescBatch {
    SolveDesc d[4];
};

__global__ void k_write_descs(DescBatch b, int n, SolveDesc* dev) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (threadIdx.x == 0 && i < n) dev[i] = b.d[i];
}

// ------------------------------------------- scratch of the no-alloc stepper

// Workspace of dg_rk_step_noalloc: one array per GPU, loaded with the code
// object.  Host code never passes the array's name to a kernel or a copy (on
// the host it is a stand-in, not a device address); it uses the address that
// scratch_setup looks up per device.
static __device__ __align__(256) unsigned char scratch[DG_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
    return hipSuccess;
}

void* scratch_device_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// ------------------------------------------------------------ host launchers

hipError_t upload_basis_tables(const BasisTab* host_tabs) {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_basis), host_tabs, sizeof(BasisTab) * DG_MAX_ORDER);
}

hipError_t launch_write_descs(const SolveDesc* host, int n, SolveDesc* dev, hipStream_t st) {
    if (n < 1 || n > 4) return hipErrorInvalidValue;
    DescBatch b;
    for (int i = 0; i < 4; ++i) b.d[i] = host[i < n ? i : 0];
    hipLaunchKernelGGL(k_write_descs, dim3(1), dim3(64), 0, st, b, n, dev);
    return hipGetLastError();
}

#define DG_DISPATCH_PP(PPV, CALL)           \
    switch (PPV) {                          \
        case 2: { constexpr int PP = 2; CALL; } break; \
        case 3: { constexpr int PP = 3; CALL; } break; \
        case 4: { constexpr int PP = 4; CALL; } break; \
        case 5: { constexpr int PP = 5; CALL; } break; \
        case 6: { constexpr int PP = 6; CALL; } break; \
        case 7: { constexpr int PP = 7; CALL; } break; \
        case 8: { constexpr int PP = 8; CALL; } break; \
        case 9: { constexpr int PP = 9; CALL; } break; \
        default: return hipErrorInvalidValue;          \
    }

hipError_t launch_traces(int PPv, const DescList& dl, hipStream_t st) {
    const int nb = dl.blk[dl.n];
    DG_DISPATCH_PP(PPv, hipLaunchKernelGGL(k_traces<PP>, dim3(nb), dim3(Shape<PP>::NT), 0, st, dl));
    return hipGetLastError();
}

hipError_t launch_grad(int PPv, const DescList& dl, hipStream_t st) {
    const int nb = dl.blk[dl.n];
    if (dl.n == 1 && dl.inl) {
        DG_DISPATCH_PP(PPv, hipLaunchKernelGGL(k_grad1<PP>, dim3(nb), dim3(Shape<PP>::NT), 0, st, dl));
        return hipGetLastError();
    }
    DG_DISPATCH_PP(PPv, hipLaunchKernelGGL(k_grad<PP>, dim3(nb), dim3(Shape<PP>::NT), 0, st, dl));
    return hipGetLastError();
}

// compute units of the current device (persistent launches size their grid
// by it), looked up once per device
int cu_count() {
    static std::mutex mu;
    static int cus[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (cus[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

hipError_t launch_grad_net(int PPv, const DescList& dl, const NetArgs& na, const NetTarget& T, hipStream_t st) {
    if (PPv != 4 || dl.n != 1 || !dl.inl || T.E % kRows != 0 || na.dims[0] != na.n_in * 64) return hipErrorInvalidValue;
    int pmax = 0;
    for (int l = 0; l <= na.n_layers; ++l) pmax = pmax > na.pdims[l] ? pmax : na.pdims[l];
    const size_t smem = (size_t)kRowWaves * GradLds<4>::N * sizeof(double) +
                        (size_t)2 * kRows * (pmax + kLdPad) * sizeof(uint16_t);
    // the dynamic LDS limit, raised once per device to the largest size asked
    static std::mutex mu;
    static size_t set_for[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (set_for[dev] < smem) {
            e = hipFuncSetAttribute((const void*)k_grad_net<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            if (e != hipSuccess) return e;
            set_for[dev] = smem;
        }
    }
    hipLaunchKernelGGL(k_grad_net<4>, dim3(T.E / kRows), dim3(kRowThreads), smem, st, dl, na, T);
    return hipGetLastError();
}

hipError_t launch_resid(int PPv, int update, const DescList& dl, double rkA, double rkB, int first_stage,
                        hipStream_t st) {
    const int nb = dl.blk[dl.n];
    if (PPv == 9 && dl.n == 1) {
        // one solve at P = 8: a block per CU (the block's LDS allows no
        // second), each walking its share of the elements
        const int grid = nb < cu_count() ? nb : cu_count();
        if (update)
            hipLaunchKernelGGL((k_resid_loop<9, 1>), dim3(grid), dim3(Shape<9>::NT), 0, st, dl, rkA, rkB, first_stage);
        else
            hipLaunchKernelGGL((k_resid_loop<9, 0>), dim3(grid), dim3(Shape<9>::NT), 0, st, dl, rkA, rkB, first_stage);
        return hipGetLastError();
    }
    if (dl.n == 1 && dl.inl) {
        if (update) {
            DG_DISPATCH_PP(PPv, hipLaunchKernelGGL((k_resid1<PP, 1>), dim3(nb), dim3(Shape<PP>::NT), 0, st, dl, rkA,
                                                   rkB, first_stage));
        } else {
            DG_DISPATCH_PP(PPv, hipLaunchKernelGGL((k_resid1<PP, 0>), dim3(nb), dim3(Shape<PP>::NT), 0, st, dl, rkA,
                                                   rkB, first_stage));
        }
        return hipGetLastError();
    }
    if (update) {
        DG_DISPATCH_PP(PPv, hipLaunchKernelGGL((k_resid<PP, 1>), dim3(nb), dim3(Shape<PP>::NT), 0, st, dl, rkA, rkB,
                                               first_stage));
    } else {
        DG_DISPATCH_PP(PPv, hipLaunchKernelGGL((k_resid<PP, 0>), dim3(nb), dim3(Shape<PP>::NT), 0, st, dl, rkA, rkB,
                                               first_stage));
    }
    return hipGetLastError();
}

hipError_t launch_tgv(int PPv, const Phys& ph, int N, double* q, hipStream_t st) {
    DG_DISPATCH_PP(PPv, hipLaunchKernelGGL(k_tgv<PP>, dim3(N * N * N), dim3(Shape<PP>::NT), 0, st, ph, N, q));
    return hipGetLastError();
}

hipError_t launch_diag(int PPv, const Phys& ph, int N, const double* q, double* partial, double* out,
                       hipStream_t st) {
    const int E = N * N * N;
    DG_DISPATCH_PP(PPv, hipLaunchKernelGGL(k_diag_partial<PP>, dim3(E), dim3(256), 0, st, ph, E, q, partial));
    const double J = (ph.h * 0.5) * (ph.h * 0.5) * (ph.h * 0.5);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, E, J, partial, out);
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(64), 0, st, out, J / (ph.L * ph.L * ph.L));
    return hipGetLastError();
}

hipError_t launch_err_inf(int PPv, int E, const double* q, const double* qref, double* partial, double* out,
                          hipStream_t st) {
    const int NP = PPv * PPv * PPv;
    hipLaunchKernelGGL(k_err_partial, dim3(E), dim3(256), 0, st, E, NP, q, qref, partial);
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(256), 0, st, E, partial, out);
    return hipGetLastError();
}

template <int PPS>
static hipError_t launch_project_s(int PPd, const ProjArg& pa, int E, const double* src, double* dst, hipStream_t st) {
    switch (PPd) {
#define DG_PROJ_CASE(V)                                                                                    \
    case V:                                                                                                \
        if constexpr (V <= PPS)                                                                            \
            hipLaunchKernelGGL((k_project<PPS, V>), dim3(E), dim3(256), 0, st, pa, E, src, dst);           \
        else                                                                                               \
            return hipErrorInvalidValue;                                                                   \
        break;
        DG_PROJ_CASE(2) DG_PROJ_CASE(3) DG_PROJ_CASE(4) DG_PROJ_CASE(5) DG_PROJ_CASE(6) DG_PROJ_CASE(7)
        DG_PROJ_CASE(8) DG_PROJ_CASE(9)
#undef DG_PROJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_project(int PPs, int PPd, int E, const double* G1, const double* src, double* dst,
                          hipStream_t st) {
    ProjArg pa;
    for (int x = 0; x < PPd * PPs; ++x) pa.G[x] = G1[x];
    switch (PPs) {
        case 2: return launch_project_s<2>(PPd, pa, E, src, dst, st);
        case 3: return launch_project_s<3>(PPd, pa, E, src, dst, st);
        case 4: return launch_project_s<4>(PPd, pa, E, src, dst, st);
        case 5: return launch_project_s<5>(PPd, pa, E, src, dst, st);
        case 6: return launch_project_s<6>(PPd, pa, E, src, dst, st);
        case 7: return launch_project_s<7>(PPd, pa, E, src, dst, st);
        case 8: return launch_project_s<8>(PPd, pa, E, src, dst, st);
        case 9: return launch_project_s<9>(PPd, pa, E, src, dst, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_pairs(int E, int n_p, double div, const double* Gq, const double* GR, const double* R3,
                             float* x, float* y, hipStream_t st) {
    const size_t total = (size_t)5 * E * n_p;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_pack_pairs, dim3(blocks), dim3(256), 0, st, E, n_p, div, Gq, GR, R3, x, y);
    return hipGetLastError();
}

}  // namespace dgnn
