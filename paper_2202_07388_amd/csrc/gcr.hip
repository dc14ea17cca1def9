// gcr.hip -- flexible GCR with restarts and a variable preconditioner (paper Sec. 3.1,
// openQ*D's fgcr; settings res, nmx, nkv, ncy, nmr, bs of Table 2). The outer iteration
// and every reduction run in FP64 (ldtype = rdtype = binary64); the SAP preconditioner
// runs in the small type sdtype (FP32, FP16 or BF16 storage, FP32 arithmetic).
//
// Step k of a cycle: phi_k = M(rho); chi_k = D phi_k; Gram-Schmidt against chi_0..k-1
// with all coefficients from one fused multi-dot pass (classical GS), then one pass
// that subtracts them and forms |chi_k|^2 and chi_k^+ rho, then one pass that normalises
// chi_k and updates rho (with |rho|^2). Coefficients never leave the device within a
// cycle; the host reads |rho| per step (convergence) and the triangular factor R and c
// once per cycle, solves R alpha = c and updates psi += sum alpha_l phi_l. The restart
// step recomputes rho = eta - D psi in FP64.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "sap.h"

namespace qdw {

int nn_precondition(qdw_op* op, const void* nn, const void* rho, void* phi, double rho_norm,
                    char* work, hipStream_t st);
size_t nn_precond_workspace(const qdw_op* op);

namespace {

// a_lk = chi_l^+ v for l < K (complex), FP64
template <int K>
struct MultiDot {
    static constexpr int NS = 2 * K;
    const void* chi[kMaxKv];
    const void* v;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        cx<double> vv[4];
        ld4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            cx<double> c[4];
            ld4<F64, double>(chi[l], Vh, u.par, u.g, u.i, c);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const cx<double> z = cmul_conj(c[j], vv[j]);
                acc[2 * l] += z.re;
                acc[2 * l + 1] += z.im;
            }
        }
    }
};

// v -= sum_l a_lk chi_l ; |v|^2 ; v^+ rho
template <int K>
struct GsUpdate {
    static constexpr int NS = 3;
    const void* chi[kMaxKv];
    void* v;
    const void* rho;
    const double* a;  // a_lk at a[2l], a[2l+1]
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        cx<double> vv[4], rr[4];
        ld4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const cx<double> al = {a[2 * l], a[2 * l + 1]};
            cx<double> c[4];
            ld4<F64, double>(chi[l], Vh, u.par, u.g, u.i, c);
#pragma unroll
            for (int j = 0; j < 4; ++j) vv[j] = vv[j] - al * c[j];
        }
        if (K > 0) st4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
        ld4<F64, double>(rho, Vh, u.par, u.g, u.i, rr);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[0] += vv[j].re * vv[j].re + vv[j].im * vv[j].im;
            const cx<double> z = cmul_conj(vv[j], rr[j]);
            acc[1] += z.re;
            acc[2] += z.im;
        }
    }
};

// chi_k = v / b_k ; rho -= (c_k / b_k) v ; |rho|^2
struct GcrUpdate {
    static constexpr int NS = 1;
    void* v;
    void* rho;
    const double* coef;  // 1/b, Re c/b, Im c/b
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        const double ib = coef[0];
        const cx<double> cb = {coef[1], coef[2]};
        cx<double> vv[4], rr[4];
        ld4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
        ld4<F64, double>(rho, Vh, u.par, u.g, u.i, rr);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            rr[j] = rr[j] - cb * vv[j];
            vv[j] = scale(vv[j], ib);
            acc[0] += rr[j].re * rr[j].re + rr[j].im * rr[j].im;
        }
        st4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
        st4<F64, double>(rho, Vh, u.par, u.g, u.i, rr);
    }
};

// psi += sum_l alpha_l phi_l
template <int K>
struct MultiAxpy {
    static constexpr int NS = 0;
    void* psi;
    const void* phi[kMaxKv];
    double al[2 * kMaxKv];
    int Vh;
    __device__ void operator()(const Unit& u, double*) const
    {
        cx<double> p[4];
        ld4<F64, double>(psi, Vh, u.par, u.g, u.i, p);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const cx<double> a = {al[2 * l], al[2 * l + 1]};
            cx<double> f[4];
            ld4<F64, double>(phi[l], Vh, u.par, u.g, u.i, f);
#pragma unroll
            for (int j = 0; j < 4; ++j) p[j] = p[j] + a * f[j];
        }
        st4<F64, double>(psi, Vh, u.par, u.g, u.i, p);
    }
};

template <template <int> class F, class Fill>
int dispatch_k(int k, const qdw_op* op, hipStream_t st, Fill fill, double* out = nullptr,
               int fin = FIN_STORE, int kk = 0)
{
    switch (k) {
#define QDW_K(n)                                                                       \
    case n: {                                                                          \
        F<n> f;                                                                        \
        fill(f);                                                                       \
        return run_map(op, f, st, out, fin, kk);                                       \
    }
        QDW_K(0) QDW_K(1) QDW_K(2) QDW_K(3) QDW_K(4) QDW_K(5) QDW_K(6) QDW_K(7) QDW_K(8)
        QDW_K(9) QDW_K(10) QDW_K(11) QDW_K(12) QDW_K(13) QDW_K(14) QDW_K(15) QDW_K(16)
#undef QDW_K
    default: QDW_CHECK(false, QDW_EINVAL, "GCR: nkv above 16");
    }
}

struct GcrLayout {
    void* rho;
    void* tmp;
    void* phi[kMaxKv];
    void* chi[kMaxKv];
    double* gsc;
    char* pre;  // preconditioner workspace
};

size_t precond_bytes(const qdw_op* op, const qdw_sap_gcr_params& p)
{
    size_t b = 0;
    if (p.precond == QDW_PRECOND_SAP || p.precond == QDW_PRECOND_NN_SAP ||
        p.precond == QDW_PRECOND_SAP_ADAPTIVE || p.precond == QDW_PRECOND_SAP_EO)
        b = sap_workspace(op, p.sdtype);
    if (p.precond == QDW_PRECOND_NN || p.precond == QDW_PRECOND_NN_SAP)
        b = std::max(b, nn_precond_workspace(op));
    return b;
}

size_t layout(const qdw_op* op, const qdw_sap_gcr_params& p, char* base, GcrLayout* L)
{
    const size_t fb = spinor_bytes(op->g, F64);
    size_t off = 0;
    auto take = [&](size_t n) {
        char* at = base ? base + off : nullptr;
        off += (n + 255) & ~(size_t)255;
        return at;
    };
    L->rho = take(fb);
    L->tmp = take(fb);
    for (int k = 0; k < p.nkv; ++k) L->phi[k] = take(fb);
    for (int k = 0; k < p.nkv; ++k) L->chi[k] = take(fb);
    L->gsc = (double*)take(sizeof(double) * G_SIZE);
    L->pre = take(precond_bytes(op, p));
    return off + 256;
}

int gcr_impl(qdw_op* op, const void* eta, void* psi, const qdw_sap_gcr_params& p, char* work,
             qdw_info* info, hipStream_t st)
{
    const Geom& g = op->g;
    const int Vh = g.Vh;
    GcrLayout L;
    layout(op, p, work, &L);
    BlockGeom B{};
    int rc;
    const bool adaptive = p.precond == QDW_PRECOND_SAP_ADAPTIVE;
    const bool sap_eo = p.precond == QDW_PRECOND_SAP_EO;
    if (p.precond == QDW_PRECOND_SAP || p.precond == QDW_PRECOND_NN_SAP || adaptive || sap_eo)
        if ((rc = make_block_geom(g, p.bs, &B))) return rc;
#define TRY(x) do { if ((rc = (x)) != QDW_OK) return rc; } while (0)
    info->status = 0;
    info->nreset = 0;
    info->n_dw_hi = info->n_dw_lo = 0;
    info->n_steps = 0;
    info->rel_res_true = 0.0;
    TRY(run_map(op, Zero<F64>{psi, Vh}, st));
    TRY(run_map(op, Axpby<F64, F64>{eta, L.rho, 1.0, 0.0, Vh}, st));
    if (adaptive) TRY(sap_ctrl_reset_total(sap_ctrl(op, p.sdtype, L.pre), st));
    double eta2;
    TRY(run_map(op, Norm2<F64>{eta, Vh}, st, op->scalars + S_TMP));
    TRY(read_scalars(op, S_TMP, 1, &eta2, st));
    if (!(eta2 > 0.0)) {
        info->status = std::isfinite(eta2) ? 0 : -3;
        return QDW_OK;
    }
    const double neta = std::sqrt(eta2);
    const double tol = p.res * neta;
    double rn = neta;
    int steps = 0, status = 0;
    bool nn_ok = p.precond == QDW_PRECOND_NN || p.precond == QDW_PRECOND_NN_SAP;
    std::vector<double> hs(G_SIZE);
    while (true) {
        int k = 0;
        bool dropped = false;
        while (k < p.nkv && steps < p.nmx && rn > tol) {
            // phi_k = M(rho)
            const double rn_before = rn;
            bool use_nn = nn_ok;
            if (use_nn) {
                TRY(nn_precondition(op, p.nn_weights, L.rho, L.phi[k], rn, L.pre, st));
            } else if (p.precond == QDW_PRECOND_SAP || p.precond == QDW_PRECOND_NN_SAP ||
                       sap_eo) {
                TRY(sap_run(op, L.rho, L.phi[k], rn, p.ncy, p.nmr, B, p.sdtype, L.pre, st,
                            sap_eo));
                info->n_dw_lo += p.ncy * p.nmr;
            } else if (adaptive) {
                // block tolerance: the solve's absolute target shared among the blocks
                TRY(sap_adaptive_run(op, L.rho, L.phi[k], rn, p.ncy, p.nmr, p.sap_alpha,
                                     p.res * neta / B.nblk, B, p.sdtype, L.pre, nullptr, st));
            } else {
                TRY(run_map(op, Axpby<F64, F64>{L.rho, L.phi[k], 1.0, 0.0, Vh}, st));
            }
            // chi_k = D phi_k, orthogonalised against chi_0..k-1
            TRY(dw_launch(op, L.phi[k], L.chi[k], F64, false, st));
            ++info->n_dw_hi;
            double* ak = L.gsc + G_A + 2 * kMaxKv * k;
            if (k > 0)
                TRY(dispatch_k<MultiDot>(k, op, st, [&](auto& f) {
                    for (int l = 0; l < k; ++l) f.chi[l] = L.chi[l];
                    f.v = L.chi[k];
                    f.Vh = Vh;
                }, ak));
            TRY(dispatch_k<GsUpdate>(k, op, st, [&](auto& f) {
                for (int l = 0; l < k; ++l) f.chi[l] = L.chi[l];
                f.v = L.chi[k];
                f.rho = L.rho;
                f.a = ak;
                f.Vh = Vh;
            }, L.gsc, FIN_GCR_NORM, k));
            TRY(run_map(op, GcrUpdate{L.chi[k], L.rho, L.gsc + G_COEF, Vh}, st, L.gsc + G_NORM));
            double r2;
            TRY(read_device(op, L.gsc + G_NORM, 1, &r2, st));
            if (!std::isfinite(r2)) {
                // a non-finite preconditioner output (or step): the column is dropped, and the
                // restart below builds psi from the finite columns 0..k-1 and recomputes rho
                // from it. The network hands the rest of the solve to SAP; otherwise the
                // solve ends with status -3 and that psi.
                dropped = true;
                if (use_nn && p.precond == QDW_PRECOND_NN_SAP) nn_ok = false;
                else status = -3;
                break;
            }
            ++k;
            ++steps;
            rn = std::sqrt(r2);
            // the learned preconditioner is judged by the GCR residual itself: a step that
            // reduces |rho| by less than 1 % hands the rest of the solve to SAP
            if (use_nn && p.precond == QDW_PRECOND_NN_SAP && rn > 0.99 * rn_before) nn_ok = false;
        }
        if (k > 0 || dropped) {
            // restart step: R alpha = c, psi += sum alpha_l phi_l, rho = eta - D psi
            TRY(read_device(op, L.gsc, G_SIZE, hs.data(), st));
            std::vector<std::complex<double>> al(k);
            for (int i = k - 1; i >= 0; --i) {
                std::complex<double> s(hs[G_C + 2 * i], hs[G_C + 2 * i + 1]);
                for (int j = i + 1; j < k; ++j) {
                    // R_ij = a_ij: coefficient of chi_i in column j
                    const std::complex<double> rij(hs[G_A + 2 * (kMaxKv * j + i)],
                                                   hs[G_A + 2 * (kMaxKv * j + i) + 1]);
                    s -= rij * al[j];
                }
                // a preconditioner output with D phi_i in the span of the previous chi
                // (b_i = 0, then also c_i = 0) contributes nothing
                al[i] = hs[G_B + i] > 0.0 ? s / hs[G_B + i] : std::complex<double>(0.0, 0.0);
            }
            if (k > 0) TRY(dispatch_k<MultiAxpy>(k, op, st, [&](auto& f) {
                f.psi = psi;
                for (int l = 0; l < k; ++l) {
                    f.phi[l] = L.phi[l];
                    f.al[2 * l] = al[l].real();
                    f.al[2 * l + 1] = al[l].imag();
                }
                f.Vh = Vh;
            }));
            TRY(dw_launch(op, psi, L.tmp, F64, false, st));
            ++info->n_dw_hi;
            TRY(run_map(op, Residual{eta, L.tmp, L.rho, Vh}, st, op->scalars + S_TMP));
            double r2;
            TRY(read_scalars(op, S_TMP, 1, &r2, st));
            ++info->nreset;
            rn = std::sqrt(r2);
        }
        if (status == -3 || !std::isfinite(rn)) {
            status = -3;
            break;
        }
        if (rn <= tol) {
            status = steps;
            break;
        }
        if (steps >= p.nmx) {
            status = -1;
            break;
        }
    }
    if (adaptive) {
        // SAP work: cycles run, each counted as nmr block sweeps (an upper bound: blocks
        // may leave their MR loop early)
        int total = 0;
        QDW_HIP(hipMemcpyAsync(op->host_scalars, sap_ctrl(op, p.sdtype, L.pre) + 2, sizeof(int),
                               hipMemcpyDeviceToHost, st));
        QDW_HIP(hipStreamSynchronize(st));
        total = *(const int*)op->host_scalars;
        info->n_dw_lo = total * p.nmr;
    }
#undef TRY
    info->status = status;
    info->n_steps = steps;
    info->rel_res_true = rn / neta;
    return QDW_OK;
}

}  // namespace
}  // namespace qdw

using namespace qdw;

extern "C" size_t qdw_sap_gcr_workspace_bytes(const qdw_op* op, const qdw_sap_gcr_params* p)
{
    if (!op || !p || p->nkv < 1 || p->nkv > kMaxKv) return 0;
    GcrLayout L;
    return layout(op, *p, nullptr, &L);
}

extern "C" int sap_gcr_solve(qdw_op* op, const void* eta, void* psi, const qdw_sap_gcr_params* p,
                             void* work, size_t work_bytes, qdw_info* info, void* stream)
{
    QDW_CHECK(op && eta && psi && p && work && info, QDW_EINVAL, "sap_gcr_solve: null argument");
    QDW_CHECK(eta != psi, QDW_EINVAL, "sap_gcr_solve: eta and psi must be distinct");
    QDW_CHECK(p->nkv >= 1 && p->nkv <= kMaxKv, QDW_EINVAL, "sap_gcr_solve: need 1 <= nkv <= 16");
    QDW_CHECK(p->nmx >= 1 && p->res > 0.0, QDW_EINVAL, "sap_gcr_solve: need nmx >= 1, res > 0");
    QDW_CHECK(p->precond >= QDW_PRECOND_NONE && p->precond <= QDW_PRECOND_SAP_EO, QDW_EINVAL,
              "sap_gcr_solve: bad preconditioner");
    const bool sap = p->precond == QDW_PRECOND_SAP || p->precond == QDW_PRECOND_NN_SAP ||
                     p->precond == QDW_PRECOND_SAP_ADAPTIVE || p->precond == QDW_PRECOND_SAP_EO;
    if (p->precond == QDW_PRECOND_SAP_ADAPTIVE)
        QDW_CHECK(p->sap_alpha > 0.0, QDW_EINVAL, "sap_gcr_solve: adaptive SAP needs sap_alpha > 0");
    if (sap) {
        QDW_CHECK(p->ncy >= 0 && p->nmr >= 0, QDW_EINVAL, "sap_gcr_solve: ncy, nmr must be >= 0");
        QDW_CHECK(p->sdtype >= QDW_F32 && p->sdtype <= QDW_BF16S, QDW_EINVAL,
                  "sap_gcr_solve: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
        BlockGeom B;
        const int rc = make_block_geom(op->g, p->bs, &B);
        if (rc) return rc;
    }
    if (p->precond == QDW_PRECOND_NN || p->precond == QDW_PRECOND_NN_SAP)
        QDW_CHECK(p->nn_weights, QDW_EINVAL, "sap_gcr_solve: the NN preconditioner needs weights");
    GcrLayout L;
    QDW_CHECK(work_bytes >= layout(op, *p, nullptr, &L), QDW_EWORKSPACE,
              "sap_gcr_solve: workspace smaller than qdw_sap_gcr_workspace_bytes()");
    hipStream_t st = (hipStream_t)stream;
    char* wk = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = gcr_impl(op, eta, psi, *p, wk, info, st);
    info->t_sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}
