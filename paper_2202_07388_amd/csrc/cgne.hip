// cgne.hip -- conjugate gradient on the normal equations D^+ D psi = eta (paper Sec. 2,
// openQ*D's cgne), plain FP64 or with a low-precision inner iteration and FP64 resets.
//
// Inner iteration (precision PL for r, p, q = D p, w = D^+ q; solution correction x_lo in
// FP32, or psi itself when PL = FP64):
//     alpha = |r|^2 / |q|^2 ; x_lo += alpha p ; r -= alpha w ; beta = |r_new|^2/|r|^2 ;
//     p = r + beta p
// with every reduction in FP64 and the scalars alpha, beta kept in device memory (no
// host round trip inside an iteration). The host reads |r|^2 one iteration late, so the
// GPU never idles waiting for it.
//
// Reset step (Sec. 2 / Fig. 1: triggered once the recursive residual has dropped by an
// amount of the order of the working type's machine epsilon; it costs more than a regular
// step): psi += x_lo / s in FP64, r_hi = eta - D^+ D psi with two FP64 applications
// of D, then r = s' r_hi rounded to PL with the new scale s' = sqrt(24 V) / |r_hi|, which
// keeps FP16-stored components near unit size (Table 1: binary16 has no normal numbers
// below 6.1e-5). By default the search direction is kept (rescaled) -- a reliable update;
// keep_p = 0 restarts it from r instead.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "blas.h"

using namespace qdw;

namespace {

struct CgState {
    int steps = 0, nreset = 0, ndw_hi = 0, ndw_lo = 0, kept = 0;
};

// r = s_new r_hi (rounded to PL); sums: |r|^2 as stored, |r_hi - r_old / s_old|^2
template <int PL>
struct ResetResidual {
    static constexpr int NS = 2;
    const void* rhi;
    void* r;
    double s_old, s_new;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        cx<double> vh[4], vo[4];
        ld4<F64, double>(rhi, Vh, u.par, u.g, u.i, vh);
        ld4<PL, double>(r, Vh, u.par, u.g, u.i, vo);
        const double inv = 1.0 / s_old;
        cx<double> vn[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const cx<double> d = vh[k] - scale(vo[k], inv);
            acc[1] += d.re * d.re + d.im * d.im;
            vn[k] = scale(vh[k], s_new);
        }
        st4<PL, double>(r, Vh, u.par, u.g, u.i, vn);
        ld4<PL, double>(r, Vh, u.par, u.g, u.i, vn);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[0] += vn[k].re * vn[k].re + vn[k].im * vn[k].im;
    }
};

template <int PL, int PX>
int cgne_impl(qdw_op* op, const void* eta, void* psi, const qdw_cgne_params& prm, char* work,
              qdw_info* info, hipStream_t st)
{
    const Geom& g = op->g;
    const int Vh = g.Vh;
    const size_t f64b = spinor_bytes(g, F64), flb = spinor_bytes(g, PL);
    void* rhi = work;
    void* t1 = work + f64b;
    void* t2 = work + 2 * f64b;
    char* wp = work + 3 * f64b;
    void* xlo = psi;
    if (PL != F64) {
        xlo = wp;
        wp += spinor_bytes(g, PX);
    }
    void* r = wp;
    void* p = wp + flb;
    void* q = wp + 2 * flb;
    void* w = wp + 3 * flb;
    double* sc = op->scalars;
    const double sqrt24v = std::sqrt(24.0 * g.V);
    const double eps_inner = PL == F64 ? std::ldexp(1.0, -52) : PL == F32 ? std::ldexp(1.0, -23)
                             : PL == F16S ? std::ldexp(1.0, -10) : std::ldexp(1.0, -7);
    // default threshold: the paper's reset after a drop of about the working epsilon when
    // CG restarts; a drop of 10 between reliable updates when the direction is kept (the
    // recursive and the true residual then stay close, which keeping p requires)
    double delta = prm.delta >= 0 ? prm.delta : prm.keep_p ? 0.1 : 10.0 * eps_inner;
    if (PL == F64 && prm.delta < 0) delta = 0.0;  // FP64: check only at convergence

    // the even-odd reduced system lives on the even half of every field
    const bool schur = prm.schur != 0;
    const long nu = schur ? 3L * Vh : 0;
    auto apply = [&](const void* in, void* out, int prec, bool dag) {
        return schur ? schur_launch(op, in, out, prec, dag, st) : dw_launch(op, in, out, prec, dag, st);
    };
    CgState S;
    int rc;
#define TRY(x) do { if ((rc = (x)) != QDW_OK) return rc; } while (0)
    TRY(run_map(op, Zero<F64>{psi, Vh}, st));
    if (PL != F64) TRY(run_map(op, Zero<PX>{xlo, Vh}, st, nullptr, FIN_STORE, 0, nu));
    double eta2;
    TRY(run_map(op, Norm2<F64>{eta, Vh}, st, op->scalars + S_TMP, FIN_STORE, 0, nu));
    TRY(read_scalars(op, S_TMP, 1, &eta2, st));
    info->status = 0;
    info->nreset = 0;
    info->n_dw_hi = info->n_dw_lo = 0;
    info->rel_res_true = 0.0;
    if (!(eta2 > 0.0)) {
        info->status = std::isfinite(eta2) ? 0 : -3;
        return QDW_OK;
    }
    const double neta = std::sqrt(eta2);
    double s = PL == F64 ? 1.0 : sqrt24v / neta;
    TRY(run_map(op, ScaleNorm<F64, PL>{eta, r, s, Vh}, st, op->scalars + S_RR, FIN_STORE, 0, nu));
    TRY(run_map(op, Axpby<PL, PL>{r, p, 1.0, 0.0, Vh}, st, nullptr, FIN_STORE, 0, nu));
    double rr_reset;
    TRY(read_scalars(op, S_RR, 1, &rr_reset, st));
    double best = rr_reset, prev_true = 1.0;
    int since = 0, bad_resets = 0;
    const int stall_window = 100;

    hipEvent_t ev[2];
    QDW_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    QDW_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    double* slot = op->host_scalars + 32;

    auto iterate = [&]() -> int {
        int e;
        if ((e = apply(p, q, PL, false))) return e;
        if ((e = apply(q, w, PL, true))) return e;
        S.ndw_lo += 2;
        if ((e = run_map(op, Norm2<PL>{q, Vh}, st, op->scalars, FIN_CG_ALPHA, 0, nu))) return e;
        if ((e = run_map(op, CgStep<PX, PL>{xlo, p, r, w, sc, Vh}, st, op->scalars, FIN_CG_BETA, 0, nu))) return e;
        if ((e = run_map(op, CgDirection<PL>{r, p, sc, Vh}, st, nullptr, FIN_STORE, 0, nu))) return e;
        ++S.steps;
        const int k = S.steps & 1;
        QDW_HIP(hipMemcpyAsync(slot + k, sc + S_RR, sizeof(double), hipMemcpyDeviceToHost, st));
        QDW_HIP(hipEventRecord(ev[k], st));
        return QDW_OK;
    };

    // psi += x_lo / s ; r_hi = eta - D^+ D psi ; returns |r_hi| / |eta| in *rel. With
    // checked, x_lo is added only when it is finite (after a non-finite step).
    auto true_residual = [&](double* rel, bool checked = false) -> int {
        int e;
        bool add = PL != F64;
        if (add && checked) {
            if ((e = run_map(op, Norm2<PX>{xlo, Vh}, st, op->scalars + S_TMP, FIN_STORE, 0, nu))) return e;
            double x2;
            if ((e = read_scalars(op, S_TMP, 1, &x2, st))) return e;
            add = std::isfinite(x2);
        }
        if (add)
            if ((e = run_map(op, Accumulate<PX>{psi, xlo, 1.0 / s, Vh}, st, nullptr, FIN_STORE, 0, nu))) return e;
        if ((e = apply(psi, t1, F64, false))) return e;
        if ((e = apply(t1, t2, F64, true))) return e;
        S.ndw_hi += 2;
        if ((e = run_map(op, Residual{eta, t2, rhi, Vh}, st, op->scalars + S_TMP, FIN_STORE, 0, nu))) return e;
        double rt2;
        if ((e = read_scalars(op, S_TMP, 1, &rt2, st))) return e;
        *rel = std::sqrt(rt2) / neta;
        return QDW_OK;
    };

    // restart the inner iteration from r_hi (|r_hi| = rel * |eta|)
    auto reset = [&](double rel) -> int {
        int e;
        const double snew = PL == F64 ? 1.0 : sqrt24v / (rel * neta);
        // r = snew r_hi, with |r|^2 into S_RR and the drift |r_hi - r_old/s|^2 next to it
        if ((e = run_map(op, ResetResidual<PL>{rhi, r, s, snew, Vh}, st, op->scalars + S_RR, FIN_STORE, 0, nu))) return e;
        double d2[2];
        if ((e = read_scalars(op, S_RR, 2, d2, st))) return e;
        // keep the direction only while the recursive residual had not drifted far from
        // the true one; otherwise restart from the true residual
        const bool keep = prm.keep_p && std::sqrt(d2[1]) <= 0.3 * rel * neta;
        S.kept += keep;
        if (keep) {
            if ((e = run_map(op, Axpby<PL, PL>{p, p, snew / s, 0.0, Vh}, st, nullptr, FIN_STORE, 0, nu))) return e;
        } else {
            if ((e = run_map(op, Axpby<PL, PL>{r, p, 1.0, 0.0, Vh}, st, nullptr, FIN_STORE, 0, nu))) return e;
        }
        s = snew;
        rr_reset = d2[0];
        best = rr_reset;
        since = 0;
        ++S.nreset;
        return QDW_OK;
    };

    int status = 0;
    double rel_true = 1.0;
    bool done = false;
    TRY(iterate());
    while (!done) {
        const bool more = S.steps < prm.nmx;
        if (more) TRY(iterate());
        // value of the iteration before the one just enqueued (or the last one)
        const int k = more ? ((S.steps - 1) & 1) : (S.steps & 1);
        QDW_HIP(hipEventSynchronize(ev[k]));
        const double v = slot[k];
        if (!std::isfinite(v)) {
            QDW_HIP(hipStreamSynchronize(st));
            TRY(true_residual(&rel_true, true));
            status = -3;
            break;
        }
        if (v < 0.81 * best) {
            best = v;
            since = 0;
        } else {
            ++since;
        }
        const bool conv = std::sqrt(v) / s <= prm.res * neta;
        const bool drop = delta > 0.0 && v < delta * delta * rr_reset;
        const bool stall = since >= stall_window;
        if (conv || drop || stall || !more) {
            QDW_HIP(hipStreamSynchronize(st));
            TRY(true_residual(&rel_true));
            if (rel_true <= prm.res) {
                status = S.steps;
                break;
            }
            if (!more) {
                status = -1;
                break;
            }
            if (stall && delta == 0.0 && PL != F64) {  // no resets allowed: give up
                status = -2;
                break;
            }
            if (rel_true > 0.9 * prev_true) {
                if (++bad_resets >= 3) {
                    status = -2;
                    break;
                }
            } else {
                bad_resets = 0;
            }
            prev_true = rel_true;
            TRY(reset(rel_true));
            if (S.steps >= prm.nmx) {
                status = -1;
                break;
            }
            TRY(iterate());
        }
    }
#undef TRY
    QDW_HIP(hipStreamSynchronize(st));
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    info->status = status;
    info->nreset = S.nreset;
    info->n_dw_hi = S.ndw_hi;
    info->n_dw_lo = S.ndw_lo;
    info->rel_res_true = rel_true;
    info->n_steps = S.steps;
    return QDW_OK;
}

size_t workspace(const qdw_op* op, int inner)
{
    const Geom& g = op->g;
    size_t b = 3 * spinor_bytes(g, F64);
    if (inner != F64) b += spinor_bytes(g, F32);
    b += 4 * spinor_bytes(g, inner);
    return b + 256;
}


size_t cascade_workspace(const qdw_op* op)
{
    const size_t f = spinor_bytes(op->g, F64);
    size_t sub = std::max(workspace(op, F64), std::max(workspace(op, F32), workspace(op, BF16S)));
    return 4 * f + sub + 256;
}

int run_phase(qdw_op* op, int prec, const void* eta, void* psi, const qdw_cgne_params& prm,
              char* work, qdw_info* info, hipStream_t st)
{
    switch (prec) {
    case F64: return cgne_impl<F64, F64>(op, eta, psi, prm, work, info, st);
    case F32: return cgne_impl<F32, F32>(op, eta, psi, prm, work, info, st);
    default: return cgne_impl<BF16S, F32>(op, eta, psi, prm, work, info, st);
    }
}

// The precision cascade: defect correction with an inner CG whose storage precision rises
// BF16 -> FP32 -> FP64 as the residual passes c eps of each type.
int cascade_impl(qdw_op* op, const void* eta, void* psi, const qdw_cgne_params& prm, char* work,
                 qdw_info* info, hipStream_t st)
{
    const Geom& g = op->g;
    const int Vh = g.Vh;
    const size_t f = spinor_bytes(g, F64);
    void* rres = work;
    void* dlt = work + f;
    void* t1 = work + 2 * f;
    void* t2 = work + 3 * f;
    char* sub = work + 4 * f;
    const bool schur = prm.schur != 0;
    const long nu = schur ? 3L * Vh : 0;
    auto apply = [&](const void* in, void* out, int prec, bool dag) {
        return schur ? schur_launch(op, in, out, prec, dag, st) : dw_launch(op, in, out, prec, dag, st);
    };
    int rc;
#define TRY(x) do { if ((rc = (x)) != QDW_OK) return rc; } while (0)
    info->status = 0;
    info->nreset = 0;
    info->n_dw_hi = info->n_dw_lo = 0;
    info->n_steps = 0;
    info->rel_res_true = 0.0;
    TRY(run_map(op, Zero<F64>{psi, Vh}, st));
    TRY(run_map(op, Axpby<F64, F64>{eta, rres, 1.0, 0.0, Vh}, st, nullptr, FIN_STORE, 0, nu));
    double eta2;
    TRY(run_map(op, Norm2<F64>{eta, Vh}, st, op->scalars + S_TMP, FIN_STORE, 0, nu));
    TRY(read_scalars(op, S_TMP, 1, &eta2, st));
    if (!(eta2 > 0.0)) {
        info->status = std::isfinite(eta2) ? 0 : -3;
        return QDW_OK;
    }
    const double neta = std::sqrt(eta2);
    const double c = prm.cascade_c > 0.0 ? prm.cascade_c : 1.0;
    const struct { int prec; double tau; } phases[3] = {
        {BF16S, c * std::ldexp(1.0, -7)}, {F32, c * std::ldexp(1.0, -23)}, {F64, 0.0}};
    double rel = 1.0;
    int status = 0;
    for (const auto& ph : phases) {
        const double target = std::max(prm.res, ph.tau);
        if (rel <= target) continue;
        if (info->n_steps >= prm.nmx) {
            status = -1;
            break;
        }
        qdw_cgne_params sp = prm;
        sp.cascade = 0;
        sp.inner = (qdw_prec)ph.prec;
        sp.res = target / rel;  // relative to the current residual, the phase's source
        sp.nmx = prm.nmx - info->n_steps;
        qdw_info si{};
        TRY(run_phase(op, ph.prec, rres, dlt, sp, sub, &si, st));
        info->n_steps += si.n_steps;
        info->nreset += si.nreset;
        info->n_dw_hi += si.n_dw_hi;
        (ph.prec == F64 ? info->n_dw_hi : info->n_dw_lo) += si.n_dw_lo;
        if (si.status == -3) {
            status = -3;
            break;
        }
        // psi += delta ; residual of the whole system in FP64
        TRY(run_map(op, Axpby<F64, F64>{dlt, psi, 1.0, 1.0, Vh}, st, nullptr, FIN_STORE, 0, nu));
        TRY(apply(psi, t1, F64, false));
        TRY(apply(t1, t2, F64, true));
        info->n_dw_hi += 2;
        double r2;
        TRY(run_map(op, Residual{eta, t2, rres, Vh}, st, op->scalars + S_TMP, FIN_STORE, 0, nu));
        TRY(read_scalars(op, S_TMP, 1, &r2, st));
        rel = std::sqrt(r2) / neta;
        ++info->nreset;  // the phase switch is a reset step too
        if (!std::isfinite(rel)) {
            status = -3;
            break;
        }
        // a phase that stagnated (-2) or ran out of steps (-1) hands over to the next type
    }
#undef TRY
    if (status == 0) status = rel <= prm.res ? info->n_steps : (info->n_steps >= prm.nmx ? -1 : -2);
    info->status = status;
    info->rel_res_true = rel;
    return QDW_OK;
}

}  // namespace

extern "C" size_t qdw_cgne_workspace_bytes(const qdw_op* op, const qdw_cgne_params* prm)
{
    if (!op || !prm) return 0;
    if (prm->cascade) return cascade_workspace(op);
    if (prm->inner < QDW_F64 || prm->inner > QDW_BF16S) return 0;
    return workspace(op, prm->inner);
}

extern "C" int cgne_solve(qdw_op* op, const void* eta, void* psi, const qdw_cgne_params* prm,
                          void* work, size_t work_bytes, qdw_info* info, void* stream)
{
    QDW_CHECK(op && eta && psi && prm && work && info, QDW_EINVAL, "cgne_solve: null argument");
    QDW_CHECK(prm->cascade || (prm->inner >= QDW_F64 && prm->inner <= QDW_BF16S), QDW_EINVAL,
              "cgne_solve: bad inner precision");
    QDW_CHECK(prm->nmx >= 1 && prm->res > 0.0, QDW_EINVAL, "cgne_solve: need nmx >= 1, res > 0");
    QDW_CHECK(eta != psi, QDW_EINVAL, "cgne_solve: eta and psi must be distinct");
    QDW_CHECK(work_bytes >= (prm->cascade ? cascade_workspace(op) : workspace(op, prm->inner)),
              QDW_EWORKSPACE, "cgne_solve: workspace smaller than qdw_cgne_workspace_bytes()");
    hipStream_t st = (hipStream_t)stream;
    char* wk = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    const auto t0 = std::chrono::steady_clock::now();
    int rc;
    if (prm->cascade) {
        rc = cascade_impl(op, eta, psi, *prm, wk, info, st);
        info->t_sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return rc;
    }
    switch (prm->inner) {
    case QDW_F64: rc = cgne_impl<F64, F64>(op, eta, psi, *prm, wk, info, st); break;
    case QDW_F32: rc = cgne_impl<F32, F32>(op, eta, psi, *prm, wk, info, st); break;
    case QDW_F16S: rc = cgne_impl<F16S, F32>(op, eta, psi, *prm, wk, info, st); break;
    default: rc = cgne_impl<BF16S, F32>(op, eta, psi, *prm, wk, info, st); break;
    }
    info->t_sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}
