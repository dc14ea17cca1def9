// batch.hip -- many SAP-GCR solves at once, over lattices of different volumes, with
// several GCR restart cycles of the whole batch captured once as a single HIP graph.
//
// The solves follow the flexible GCR of the paper (Sec. 3.1, settings of Table 2) step for
// step, exactly as sap_gcr_solve runs them for one right-hand side; what changes is who
// decides. Every decision that sap_gcr_solve takes on the host (the SAP storage scale from
// |rho|, convergence after a step, the triangular solve R alpha = c at a restart, the
// end of the solve) is taken here by small device kernels that read the per-right-hand-side
// scalars and set per-right-hand-side flags. Every kernel of a step checks its right-hand
// side's flag on entry and returns at once when that solve has left the cycle, so the
// same captured sequence serves every right-hand side whatever its progress. A batch plan
// (qdw_batch) captures `cycles` restart cycles (nkv steps + the restart step each) once;
// a solve launches that graph on the caller's stream and waits once per launch, to read
// the flags, so a batch that finishes within `cycles` cycles takes one launch and one
// host wait, and the plan is reused by every later solve of the same batch shape.
//
// Right-hand sides that share an operator form a group. A group's fields are stored
// right-hand-side-fastest at a fixed byte stride and every kernel covers all of them
// (blockIdx.y or the multi-right-hand-side D kernel): the links and clover blocks of a
// tile are read once for all right-hand sides of that lattice, and one launch carries the
// whole group. Groups are independent branches of the graph, so the kernels of a small
// lattice fill the machine next to those of a large one.
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "sap.h"

namespace qdw {

int dw_launch_multi(qdw_op* op, const void* const* in, void* const* out, int nrhs, int prec,
                    bool dag, const int* gate, int gstride, hipStream_t st);

namespace {

// per-right-hand-side control flags (ints)
enum { F_ACTIVE = 0, F_INCYCLE, F_KDONE, F_STEPS, F_STATUS, F_NRESET, F_SIZE = 8 };
// per-right-hand-side doubles: the GCR block, then alpha, |eta|^2 and the absolute tolerance
enum { B_ALPHA = G_SIZE, B_ETA2 = B_ALPHA + 2 * kMaxKv, B_TOL, B_SIZE = 640 };
constexpr int kNsMax = 2 * kMaxKv;                    // widest reduction of a step
constexpr long kPartStride = (long)kMaxPartials * kNsMax;

struct Group {
    qdw_op* op;
    std::vector<int> prob;  // problem indices of this group's right-hand sides
    int nr;
    BlockGeom B;
    long fb, fbs;           // bytes per FP64 field, per storage-precision field
    char *eta, *x, *rho, *tmp, *phi, *chi;  // FP64: field (l, r) of phi at phi + (l nr + r) fb
    char *rs, *psis, *delta;                // SAP storage precision, r at rs + r fbs
    double* sc;                             // nr * B_SIZE
    int* fl;                                // nr * F_SIZE (inside one array for all groups)
    double* part;                           // nr * kPartStride
    hipStream_t s;
};

// ---------------------------------------------------------------- batched map / finalise

template <class F>
__global__ __launch_bounds__(256) void bmap_kernel(long nunits, int Vh, F f, double* partials,
                                                   const int* fl, int gate)
{
    const int r = blockIdx.y;
    if (gate >= 0 && !fl[r * F_SIZE + gate]) return;
    double acc[F::NS > 0 ? F::NS : 1];
#pragma unroll
    for (int k = 0; k < (F::NS > 0 ? F::NS : 1); ++k) acc[k] = 0.0;
    for (long u = (long)blockIdx.x * blockDim.x + threadIdx.x; u < nunits;
         u += (long)gridDim.x * blockDim.x)
        f(unit_of(u, Vh), acc, r);
    if constexpr (F::NS > 0)
        block_reduce_store<F::NS>(acc, partials + r * kPartStride + (long)blockIdx.x * F::NS);
}

__global__ __launch_bounds__(256) void bfinalize_kernel(const double* partials, int nblk, int ns,
                                                        double* sc, int off, int op, int k,
                                                        const int* fl, int gate)
{
    const int r = blockIdx.x;
    if (gate >= 0 && !fl[r * F_SIZE + gate]) return;
    finalize_body(partials + r * kPartStride, nblk, ns, sc + (long)r * B_SIZE + off, op, k);
}

// launch f over every right-hand side of group G (gate: flag that must be set, or -1);
// with F::NS > 0 the sums go through scalar program fin into sc[r][off ...]
template <class F>
int brun(const Group& G, const F& f, int gate, hipStream_t st, int off = 0, int fin = FIN_STORE,
         int k = 0)
{
    const long nunits = 3L * G.op->g.V;
    const int nb = map_blocks(nunits);
    bmap_kernel<F><<<dim3(nb, G.nr), 256, 0, st>>>(nunits, G.op->g.Vh, f, G.part, G.fl, gate);
    QDW_LAUNCH_CHECK();
    if constexpr (F::NS > 0) {
        bfinalize_kernel<<<G.nr, 256, 0, st>>>(G.part, nb, F::NS, G.sc, off, fin, k, G.fl, gate);
        QDW_LAUNCH_CHECK();
    }
    return QDW_OK;
}

// ---------------------------------------------------------------- functors (right-hand side r)

struct Fld {
    char* base;
    long stride;
    __device__ void* at(int r) const { return base + r * stride; }
};

// x = 0 ; rho = eta ; |eta|^2
struct Init {
    static constexpr int NS = 1;
    Fld eta, x, rho;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc, int r) const
    {
        cx<double> e[4];
        const cx<double> z[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        ld4<F64, double>(eta.at(r), Vh, u.par, u.g, u.i, e);
        st4<F64, double>(x.at(r), Vh, u.par, u.g, u.i, z);
        st4<F64, double>(rho.at(r), Vh, u.par, u.g, u.i, e);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[0] += e[j].re * e[j].re + e[j].im * e[j].im;
    }
};

__device__ __forceinline__ double sap_scale(const double* sc, int V)
{
    const double rn = sqrt(sc[G_NORM]);
    return rn > 0.0 ? sqrt(24.0 * V) / rn : 0.0;
}

// rs = s rho (rounded to the storage precision), psis = 0; s = sqrt(24 V) / |rho|
template <int SP>
struct SapIn {
    static constexpr int NS = 0;
    Fld rho, rs, psis;
    const double* sc;
    int Vh, V;
    __device__ void operator()(const Unit& u, double*, int r) const
    {
        const double s = sap_scale(sc + (long)r * B_SIZE, V);
        cx<double> v[4];
        const cx<double> z[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        ld4<F64, double>(rho.at(r), Vh, u.par, u.g, u.i, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = scale(v[j], s);
        st4<SP, double>(rs.at(r), Vh, u.par, u.g, u.i, v);
        st4<SP, double>(psis.at(r), Vh, u.par, u.g, u.i, z);
    }
};

// phi = psis / s (binary32 product, as the single-solve path forms it)
template <int SP>
struct SapOut {
    static constexpr int NS = 0;
    Fld psis, phi;
    const double* sc;
    int Vh, V;
    __device__ void operator()(const Unit& u, double*, int r) const
    {
        const float a = (float)(1.0 / sap_scale(sc + (long)r * B_SIZE, V));
        cx<float> v[4];
        ld4<SP, float>(psis.at(r), Vh, u.par, u.g, u.i, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = scale(v[j], a);
        st4<F64, float>(phi.at(r), Vh, u.par, u.g, u.i, v);
    }
};

// phi = rho (no preconditioner)
struct Copy {
    static constexpr int NS = 0;
    Fld src, dst;
    int Vh;
    __device__ void operator()(const Unit& u, double*, int r) const
    {
        cx<double> v[4];
        ld4<F64, double>(src.at(r), Vh, u.par, u.g, u.i, v);
        st4<F64, double>(dst.at(r), Vh, u.par, u.g, u.i, v);
    }
};

// a_lk = chi_l^+ chi_k, l < K
template <int K>
struct BMultiDot {
    static constexpr int NS = 2 * K;
    Fld chi;  // chi_l for right-hand side r at base + (l nr + r) stride
    int nr, k, Vh;
    __device__ void operator()(const Unit& u, double* acc, int r) const
    {
        cx<double> vv[4];
        ld4<F64, double>(chi.at(k * nr + r), Vh, u.par, u.g, u.i, vv);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            cx<double> c[4];
            ld4<F64, double>(chi.at(l * nr + r), Vh, u.par, u.g, u.i, c);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const cx<double> z = cmul_conj(c[j], vv[j]);
                acc[2 * l] += z.re;
                acc[2 * l + 1] += z.im;
            }
        }
    }
};

// chi_k -= sum_l a_lk chi_l ; |chi_k|^2 ; chi_k^+ rho
template <int K>
struct BGsUpdate {
    static constexpr int NS = 3;
    Fld chi, rho;
    const double* sc;
    int nr, Vh;
    __device__ void operator()(const Unit& u, double* acc, int r) const
    {
        const double* a = sc + (long)r * B_SIZE + G_A + 2 * kMaxKv * K;
        void* v = chi.at(K * nr + r);
        cx<double> vv[4], rr[4];
        ld4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const cx<double> al = {a[2 * l], a[2 * l + 1]};
            cx<double> c[4];
            ld4<F64, double>(chi.at(l * nr + r), Vh, u.par, u.g, u.i, c);
#pragma unroll
            for (int j = 0; j < 4; ++j) vv[j] = vv[j] - al * c[j];
        }
        if (K > 0) st4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
        ld4<F64, double>(rho.at(r), Vh, u.par, u.g, u.i, rr);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[0] += vv[j].re * vv[j].re + vv[j].im * vv[j].im;
            const cx<double> z = cmul_conj(vv[j], rr[j]);
            acc[1] += z.re;
            acc[2] += z.im;
        }
    }
};

// chi_k = chi_k / b_k ; rho -= (c_k / b_k) chi_k ; |rho|^2
struct BGcrUpdate {
    static constexpr int NS = 1;
    Fld chi, rho;
    const double* sc;
    int nr, k, Vh;
    __device__ void operator()(const Unit& u, double* acc, int r) const
    {
        const double* coef = sc + (long)r * B_SIZE + G_COEF;
        const double ib = coef[0];
        const cx<double> cb = {coef[1], coef[2]};
        void* v = chi.at(k * nr + r);
        cx<double> vv[4], rr[4];
        ld4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
        ld4<F64, double>(rho.at(r), Vh, u.par, u.g, u.i, rr);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            rr[j] = rr[j] - cb * vv[j];
            vv[j] = scale(vv[j], ib);
            acc[0] += rr[j].re * rr[j].re + rr[j].im * rr[j].im;
        }
        st4<F64, double>(v, Vh, u.par, u.g, u.i, vv);
        st4<F64, double>(rho.at(r), Vh, u.par, u.g, u.i, rr);
    }
};

// x += sum_{l < kdone} alpha_l phi_l
struct BMultiAxpy {
    static constexpr int NS = 0;
    Fld x, phi;
    const double* sc;
    const int* fl;
    int nr, Vh;
    __device__ void operator()(const Unit& u, double*, int r) const
    {
        const double* al = sc + (long)r * B_SIZE + B_ALPHA;
        const int kk = fl[r * F_SIZE + F_KDONE];
        cx<double> p[4];
        ld4<F64, double>(x.at(r), Vh, u.par, u.g, u.i, p);
        for (int l = 0; l < kk; ++l) {
            const cx<double> a = {al[2 * l], al[2 * l + 1]};
            cx<double> f[4];
            ld4<F64, double>(phi.at(l * nr + r), Vh, u.par, u.g, u.i, f);
#pragma unroll
            for (int j = 0; j < 4; ++j) p[j] = p[j] + a * f[j];
        }
        st4<F64, double>(x.at(r), Vh, u.par, u.g, u.i, p);
    }
};

// rho = eta - t ; |rho|^2
struct BResidual {
    static constexpr int NS = 1;
    Fld eta, t, rho;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc, int r) const
    {
        cx<double> ve[4], vt[4];
        ld4<F64, double>(eta.at(r), Vh, u.par, u.g, u.i, ve);
        ld4<F64, double>(t.at(r), Vh, u.par, u.g, u.i, vt);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ve[j] = ve[j] - vt[j];
            acc[0] += ve[j].re * ve[j].re + ve[j].im * ve[j].im;
        }
        st4<F64, double>(rho.at(r), Vh, u.par, u.g, u.i, ve);
    }
};

// ---------------------------------------------------------------- control kernels (one lane per rhs)

// after the initial residual: tolerance and flags
__global__ void init_ctrl_kernel(int* fl, double* sc, int nr, double res)
{
    const int r = threadIdx.x;
    if (r >= nr) return;
    int* f = fl + r * F_SIZE;
    double* s = sc + (long)r * B_SIZE;
    const double eta2 = s[B_ETA2];
    f[F_KDONE] = f[F_STEPS] = f[F_NRESET] = 0;
    s[G_NORM] = eta2;
    if (!(eta2 > 0.0)) {
        f[F_STATUS] = isfinite(eta2) ? 0 : -3;
        f[F_ACTIVE] = f[F_INCYCLE] = 0;
        s[B_TOL] = 0.0;
        return;
    }
    s[B_TOL] = res * sqrt(eta2);
    f[F_STATUS] = 0;
    f[F_ACTIVE] = f[F_INCYCLE] = 1;
}

// after step k of a cycle: count it, leave the cycle on convergence, nmx or a non-finite value
__global__ void step_ctrl_kernel(int* fl, const double* sc, int nr, int nmx)
{
    const int r = threadIdx.x;
    if (r >= nr) return;
    int* f = fl + r * F_SIZE;
    if (!f[F_INCYCLE]) return;
    const double* s = sc + (long)r * B_SIZE;
    ++f[F_KDONE];
    ++f[F_STEPS];
    const double r2 = s[G_NORM];
    if (!isfinite(r2)) {
        f[F_STATUS] = -3;
        f[F_INCYCLE] = 0;
        return;
    }
    if (!(sqrt(r2) > s[B_TOL]) || f[F_STEPS] >= nmx) f[F_INCYCLE] = 0;
}

// restart step, part 1: back-substitution R alpha = c over the kdone steps of the cycle
__global__ void tri_kernel(const int* fl, double* sc, int nr)
{
#pragma clang fp contract(off)
    const int r = threadIdx.x;
    if (r >= nr) return;
    const int* f = fl + r * F_SIZE;
    if (!f[F_ACTIVE]) return;
    double* s = sc + (long)r * B_SIZE;
    const int k = f[F_KDONE];
    double* al = s + B_ALPHA;
    for (int i = k - 1; i >= 0; --i) {
        double re = s[G_C + 2 * i], im = s[G_C + 2 * i + 1];
        for (int j = i + 1; j < k; ++j) {
            // R_ij = a_ij: coefficient of chi_i in column j
            const double rr = s[G_A + 2 * (kMaxKv * j + i)], ri = s[G_A + 2 * (kMaxKv * j + i) + 1];
            const double pr = rr * al[2 * j] - ri * al[2 * j + 1];
            const double pi = rr * al[2 * j + 1] + ri * al[2 * j];
            re -= pr;
            im -= pi;
        }
        // a preconditioner output with D phi_i in the span of the previous chi contributes 0
        const double b = s[G_B + i];
        al[2 * i] = b > 0.0 ? re / b : 0.0;
        al[2 * i + 1] = b > 0.0 ? im / b : 0.0;
    }
}

// restart step, part 2: after rho = eta - D x, decide the solve's fate
__global__ void restart_ctrl_kernel(int* fl, const double* sc, int nr, int nmx)
{
    const int r = threadIdx.x;
    if (r >= nr) return;
    int* f = fl + r * F_SIZE;
    if (!f[F_ACTIVE]) return;
    const double* s = sc + (long)r * B_SIZE;
    ++f[F_NRESET];
    const double rn = sqrt(s[G_NORM]);
    f[F_KDONE] = 0;
    if (f[F_STATUS] == -3 || !isfinite(rn)) {
        f[F_STATUS] = -3;
        f[F_ACTIVE] = f[F_INCYCLE] = 0;
    } else if (!(rn > s[B_TOL])) {
        f[F_STATUS] = f[F_STEPS];
        f[F_ACTIVE] = f[F_INCYCLE] = 0;
    } else if (f[F_STEPS] >= nmx) {
        f[F_STATUS] = -1;
        f[F_ACTIVE] = f[F_INCYCLE] = 0;
    } else {
        f[F_INCYCLE] = 1;
    }
}

// ---------------------------------------------------------------- one cycle of one group

template <template <int> class F, class Fill>
int by_k(int k, Fill fill)
{
    switch (k) {
#define QDW_K(n) case n: { F<n> f; return fill(f); }
        QDW_K(0) QDW_K(1) QDW_K(2) QDW_K(3) QDW_K(4) QDW_K(5) QDW_K(6) QDW_K(7) QDW_K(8)
        QDW_K(9) QDW_K(10) QDW_K(11) QDW_K(12) QDW_K(13) QDW_K(14) QDW_K(15)
#undef QDW_K
    default: QDW_CHECK(false, QDW_EINVAL, "GCR: nkv above 16");
    }
}

// SAP (plain or with even-odd reduced block solves) with at least one cycle
inline bool sap_precond(const qdw_sap_gcr_params& p)
{
    return (p.precond == QDW_PRECOND_SAP || p.precond == QDW_PRECOND_SAP_EO) && p.ncy > 0;
}

template <int SP>
int precondition(const Group& G, const qdw_sap_gcr_params& p, void* phi_k, hipStream_t st)
{
    const int Vh = G.op->g.Vh, V = G.op->g.V;
    int rc;
    if ((rc = brun(G, SapIn<SP>{{G.rho, G.fb}, {G.rs, G.fbs}, {G.psis, G.fbs}, G.sc, Vh, V},
                   F_INCYCLE, st)))
        return rc;
    RhsStride bat;
    bat.fstride = G.fbs;
    bat.gate = G.fl + F_INCYCLE;
    bat.gstride = F_SIZE;
    if ((rc = sap_cycles(G.op, G.B, SP, p.ncy, p.nmr, G.rs, G.psis, G.delta, bat, G.nr, st,
                         p.precond == QDW_PRECOND_SAP_EO)))
        return rc;
    return brun(G, SapOut<SP>{{G.psis, G.fbs}, {(char*)phi_k, G.fb}, G.sc, Vh, V}, F_INCYCLE, st);
}

int cycle(const Group& G, const qdw_sap_gcr_params& p, hipStream_t st)
{
    const int Vh = G.op->g.Vh, nr = G.nr;
    const bool sap = sap_precond(p);
    const void* in[kMaxRhs];
    void* out[kMaxRhs];
    int rc;
    for (int k = 0; k < p.nkv; ++k) {
        char* phik = G.phi + (long)k * nr * G.fb;
        char* chik = G.chi + (long)k * nr * G.fb;
        if (sap) {
            switch (p.sdtype) {
            case QDW_F32: rc = precondition<F32>(G, p, phik, st); break;
            case QDW_F16S: rc = precondition<F16S>(G, p, phik, st); break;
            default: rc = precondition<BF16S>(G, p, phik, st); break;
            }
        } else {
            rc = brun(G, Copy{{G.rho, G.fb}, {phik, G.fb}, Vh}, F_INCYCLE, st);
        }
        if (rc) return rc;
        for (int r = 0; r < nr; ++r) {
            in[r] = phik + r * G.fb;
            out[r] = chik + r * G.fb;
        }
        if ((rc = dw_launch_multi(G.op, in, out, nr, F64, false, G.fl + F_INCYCLE, F_SIZE, st)))
            return rc;
        if (k > 0 && (rc = by_k<BMultiDot>(k, [&](auto& f) {
                f.chi = {G.chi, G.fb};
                f.nr = nr;
                f.k = k;
                f.Vh = Vh;
                return brun(G, f, F_INCYCLE, st, G_A + 2 * kMaxKv * k);
            })))
            return rc;
        if ((rc = by_k<BGsUpdate>(k, [&](auto& f) {
                f.chi = {G.chi, G.fb};
                f.rho = {G.rho, G.fb};
                f.sc = G.sc;
                f.nr = nr;
                f.Vh = Vh;
                return brun(G, f, F_INCYCLE, st, 0, FIN_GCR_NORM, k);
            })))
            return rc;
        if ((rc = brun(G, BGcrUpdate{{G.chi, G.fb}, {G.rho, G.fb}, G.sc, nr, k, Vh}, F_INCYCLE, st,
                       G_NORM)))
            return rc;
        step_ctrl_kernel<<<1, 64, 0, st>>>(G.fl, G.sc, nr, p.nmx);
        QDW_LAUNCH_CHECK();
    }
    // restart step: x += sum alpha_l phi_l ; rho = eta - D x
    tri_kernel<<<1, 64, 0, st>>>(G.fl, G.sc, nr);
    QDW_LAUNCH_CHECK();
    if ((rc = brun(G, BMultiAxpy{{G.x, G.fb}, {G.phi, G.fb}, G.sc, G.fl, nr, Vh}, F_ACTIVE, st)))
        return rc;
    for (int r = 0; r < nr; ++r) {
        in[r] = G.x + r * G.fb;
        out[r] = G.tmp + r * G.fb;
    }
    if ((rc = dw_launch_multi(G.op, in, out, nr, F64, false, G.fl + F_ACTIVE, F_SIZE, st)))
        return rc;
    if ((rc = brun(G, BResidual{{G.eta, G.fb}, {G.tmp, G.fb}, {G.rho, G.fb}, Vh}, F_ACTIVE, st,
                   G_NORM)))
        return rc;
    restart_ctrl_kernel<<<1, 64, 0, st>>>(G.fl, G.sc, nr, p.nmx);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

// ---------------------------------------------------------------- layout

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// groups of the batch (right-hand sides sharing an operator) and, with base != null, the
// pointers into the workspace; returns the bytes needed
int plan(qdw_op* const* ops, int n, const qdw_sap_gcr_params& p, char* base,
         std::vector<Group>* out, size_t* bytes)
{
    std::vector<Group>& gs = *out;
    gs.clear();
    for (int j = 0; j < n; ++j) {
        QDW_CHECK(ops[j], QDW_EINVAL, "sap_gcr_solve_batched: null operator");
        Group* G = nullptr;
        for (Group& h : gs)
            if (h.op == ops[j]) G = &h;
        if (!G) {
            gs.push_back(Group{});
            G = &gs.back();
            G->op = ops[j];
        }
        G->prob.push_back(j);
        QDW_CHECK((int)G->prob.size() <= kMaxRhs, QDW_EINVAL,
                  "sap_gcr_solve_batched: at most 64 right-hand sides per operator");
    }
    const bool sap = sap_precond(p);
    size_t off = 0;
    auto take = [&](size_t nb) {
        char* at = base ? base + off : nullptr;
        off += align256(nb);
        return at;
    };
    // flags of all groups in one array, so one copy reads them
    int nflags = 0;
    for (Group& G : gs) nflags += (int)G.prob.size() * F_SIZE;
    int* flags = (int*)take(sizeof(int) * nflags);
    int fo = 0;
    for (Group& G : gs) {
        G.nr = (int)G.prob.size();
        G.fb = (long)spinor_bytes(G.op->g, F64);
        G.fbs = sap ? (long)spinor_bytes(G.op->g, p.sdtype) : 0;
        if (sap) {
            const int rc = make_block_geom(G.op->g, p.bs, &G.B);
            if (rc) return rc;
        }
        const size_t f = (size_t)G.fb * G.nr;
        G.eta = take(f);
        G.x = take(f);
        G.rho = take(f);
        G.tmp = take(f);
        G.phi = take(f * p.nkv);
        G.chi = take(f * p.nkv);
        G.rs = sap ? take((size_t)G.fbs * G.nr) : nullptr;
        G.psis = sap ? take((size_t)G.fbs * G.nr) : nullptr;
        G.delta = sap ? take((size_t)G.fbs * G.nr) : nullptr;
        G.sc = (double*)take(sizeof(double) * B_SIZE * G.nr);
        G.part = (double*)take(sizeof(double) * kPartStride * G.nr);
        G.fl = flags ? flags + fo : nullptr;
        fo += G.nr * F_SIZE;
        G.s = nullptr;
    }
    *bytes = off + 256;
    return QDW_OK;
}

int check_params(const qdw_sap_gcr_params* p)
{
    QDW_CHECK(p->nkv >= 1 && p->nkv <= kMaxKv, QDW_EINVAL, "sap_gcr_solve_batched: need 1 <= nkv <= 16");
    QDW_CHECK(p->nmx >= 1 && p->res > 0.0, QDW_EINVAL, "sap_gcr_solve_batched: need nmx >= 1, res > 0");
    QDW_CHECK(p->precond == QDW_PRECOND_NONE || p->precond == QDW_PRECOND_SAP ||
                  p->precond == QDW_PRECOND_SAP_EO,
              QDW_EINVAL,
              "sap_gcr_solve_batched: preconditioner must be QDW_PRECOND_NONE, QDW_PRECOND_SAP "
              "or QDW_PRECOND_SAP_EO");
    if (p->precond != QDW_PRECOND_NONE) {
        QDW_CHECK(p->ncy >= 0 && p->nmr >= 0, QDW_EINVAL, "sap_gcr_solve_batched: ncy, nmr must be >= 0");
        QDW_CHECK(p->sdtype >= QDW_F32 && p->sdtype <= QDW_BF16S, QDW_EINVAL,
                  "sap_gcr_solve_batched: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    }
    return QDW_OK;
}

}  // namespace
}  // namespace qdw

using namespace qdw;

// A captured batch: its groups carved out of the caller's workspace, the HIP streams and
// events used to capture the groups as parallel branches, and the instantiated graph of
// `cycles` restart cycles of every group.
struct qdw_batch {
    std::vector<Group> gs;
    qdw_sap_gcr_params p;
    std::vector<qdw_op*> ops;
    int n = 0, cycles = 0, device = 0, nflags = 0;
    int* fl0 = nullptr;             // the flags of all groups form one array starting here
    hipStream_t cs = nullptr;       // capture stream
    std::vector<hipStream_t> side;  // one per group (capture only)
    std::vector<hipEvent_t> ev;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double capture_ms = 0.0;
    ~qdw_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipStream_t x : side) (void)hipStreamDestroy(x);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

extern "C" size_t qdw_sap_gcr_batched_workspace_bytes(qdw_op* const* ops, int n,
                                                      const qdw_sap_gcr_params* p)
{
    if (!ops || !p || n < 1 || check_params(p)) return 0;
    std::vector<Group> gs;
    size_t bytes = 0;
    if (plan(ops, n, *p, nullptr, &gs, &bytes)) return 0;
    return bytes;
}

extern "C" int qdw_batch_create(qdw_op* const* ops, int n, const qdw_sap_gcr_params* p,
                                int cycles, void* work, size_t work_bytes, qdw_batch** out)
{
    QDW_CHECK(ops && p && work && out, QDW_EINVAL, "qdw_batch_create: null argument");
    *out = nullptr;
    QDW_CHECK(n >= 1, QDW_EINVAL, "qdw_batch_create: need n >= 1");
    QDW_CHECK(cycles >= 1 && cycles <= 64, QDW_EINVAL, "qdw_batch_create: need 1 <= cycles <= 64");
    int rc = check_params(p);
    if (rc) return rc;
    for (int j = 0; j < n; ++j)
        QDW_CHECK(ops[j] && ops[j]->device == ops[0]->device, QDW_EINVAL,
                  "qdw_batch_create: all operators must live on one device");
    std::vector<Group> gs;
    size_t need = 0;
    if ((rc = plan(ops, n, *p, nullptr, &gs, &need))) return rc;
    QDW_CHECK(work_bytes >= need, QDW_EWORKSPACE,
              "qdw_batch_create: workspace smaller than qdw_sap_gcr_batched_workspace_bytes()");
    char* wk = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);

    qdw_batch* b = new qdw_batch();
    std::unique_ptr<qdw_batch> guard(b);
    if ((rc = plan(ops, n, *p, wk, &b->gs, &need))) return rc;
    b->p = *p;
    b->n = n;
    b->cycles = cycles;
    b->device = ops[0]->device;
    b->ops.assign(ops, ops + n);
    b->nflags = n * F_SIZE;
    b->fl0 = b->gs[0].fl;
    for (const Group& G : b->gs) b->fl0 = std::min(b->fl0, G.fl);

    const auto tg0 = std::chrono::steady_clock::now();
    QDW_HIP(hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking));
    b->ev.resize(b->gs.size() + 1);
    for (hipEvent_t& e : b->ev) QDW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->side.resize(b->gs.size());
    for (size_t q = 0; q < b->gs.size(); ++q) {
        QDW_HIP(hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking));
        b->gs[q].s = b->side[q];
    }
    // every group is one branch of the graph: `cycles` restart cycles one after another
    // (the groups are independent, so they meet only at the end)
    QDW_HIP(hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
    int crc = QDW_OK;
    if (hipEventRecord(b->ev[0], b->cs) != hipSuccess) crc = QDW_EDEVICE;
    for (size_t q = 0; q < b->gs.size() && !crc; ++q) {
        if (hipStreamWaitEvent(b->gs[q].s, b->ev[0], 0) != hipSuccess) {
            crc = QDW_EDEVICE;
            break;
        }
        for (int c = 0; c < cycles && !crc; ++c) crc = cycle(b->gs[q], *p, b->gs[q].s);
        if (!crc && hipEventRecord(b->ev[1 + q], b->gs[q].s) != hipSuccess) crc = QDW_EDEVICE;
        if (!crc && hipStreamWaitEvent(b->cs, b->ev[1 + q], 0) != hipSuccess) crc = QDW_EDEVICE;
    }
    const hipError_t ce = hipStreamEndCapture(b->cs, &b->graph);
    if (crc) return crc;
    QDW_HIP(ce);
    QDW_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->capture_ms = 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - tg0).count();
    *out = guard.release();
    return QDW_OK;
}

extern "C" double qdw_batch_capture_ms(const qdw_batch* b) { return b ? b->capture_ms : 0.0; }

extern "C" int qdw_batch_destroy(qdw_batch* b)
{
    if (!b) return QDW_OK;
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    delete b;
    return QDW_OK;
}

extern "C" int qdw_batch_solve(qdw_batch* b, const void* const* etas, void* const* psis,
                               qdw_info* infos, int* launches, void* stream)
{
    QDW_CHECK(b && etas && psis && infos, QDW_EINVAL, "qdw_batch_solve: null argument");
    const int n = b->n;
    for (int j = 0; j < n; ++j) {
        QDW_CHECK(etas[j] && psis[j], QDW_EINVAL, "qdw_batch_solve: null field");
        for (int q = 0; q < n; ++q)
            QDW_CHECK(psis[j] != etas[q] && (q == j || psis[j] != psis[q]), QDW_EINVAL,
                      "qdw_batch_solve: solution fields must be distinct from each other and "
                      "from every source");
    }
    int rc;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    // set-up: gather the sources, x = 0, rho = eta, |eta|^2, tolerances and flags
    for (const Group& G : b->gs) {
        for (int r = 0; r < G.nr; ++r)
            if ((rc = run_map(G.op, Axpby<F64, F64>{etas[G.prob[r]], G.eta + r * G.fb, 1.0, 0.0,
                                                    G.op->g.Vh},
                              st)))
                return rc;
        if ((rc = brun(G, Init{{G.eta, G.fb}, {G.x, G.fb}, {G.rho, G.fb}, G.op->g.Vh}, -1, st,
                       B_ETA2)))
            return rc;
        init_ctrl_kernel<<<1, 64, 0, st>>>(G.fl, G.sc, G.nr, b->p.res);
        QDW_LAUNCH_CHECK();
    }
    // the captured cycles, launched on the caller's stream until every solve has finished:
    // one launch (and one host wait) when `cycles` cycles suffice
    std::vector<int> flags(b->nflags);
    int nl = 0;
    const int max_launches = b->p.nmx / (b->cycles * 1) + 2;
    for (;;) {
        QDW_HIP(hipGraphLaunch(b->exec, st));
        ++nl;
        QDW_HIP(hipMemcpyAsync(flags.data(), b->fl0, sizeof(int) * b->nflags,
                               hipMemcpyDeviceToHost, st));
        QDW_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int q = 0; q < n; ++q) any = any || flags[q * F_SIZE + F_ACTIVE];
        if (!any) break;
        // every cycle either takes a step of each active solve or ends it
        QDW_CHECK(nl <= max_launches, QDW_EDEVICE, "qdw_batch_solve: solve did not terminate");
    }
    // results: copy the solutions out, read the per-solve outcome
    std::vector<double> hsc;
    for (const Group& G : b->gs) {
        for (int r = 0; r < G.nr; ++r)
            if ((rc = run_map(G.op, Axpby<F64, F64>{G.x + r * G.fb, psis[G.prob[r]], 1.0, 0.0,
                                                    G.op->g.Vh},
                              st)))
                return rc;
    }
    const bool sap = sap_precond(b->p);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (const Group& G : b->gs) {
        hsc.resize((size_t)B_SIZE * G.nr);
        QDW_HIP(hipMemcpyAsync(hsc.data(), G.sc, sizeof(double) * B_SIZE * G.nr,
                               hipMemcpyDeviceToHost, st));
        QDW_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < G.nr; ++r) {
            const int j = G.prob[r];
            const int* f = flags.data() + (G.fl - b->fl0) + r * F_SIZE;
            const double* sr = hsc.data() + (size_t)r * B_SIZE;
            qdw_info& in = infos[j];
            in.status = f[F_STATUS];
            in.n_steps = f[F_STEPS];
            in.nreset = f[F_NRESET];
            in.n_dw_hi = f[F_STEPS] + f[F_NRESET];
            in.n_dw_lo = sap ? (long)f[F_STEPS] * b->p.ncy * b->p.nmr : 0;
            in.rel_res_true = sr[B_ETA2] > 0.0 ? std::sqrt(sr[G_NORM] / sr[B_ETA2]) : 0.0;
            in.t_sec = secs;
        }
    }
    if (launches) *launches = nl;
    return QDW_OK;
}

extern "C" int sap_gcr_solve_batched(qdw_op* const* ops, const void* const* etas,
                                     void* const* psis, int n, const qdw_sap_gcr_params* p,
                                     void* work, size_t work_bytes, qdw_info* infos,
                                     double* graph_ms, void* stream)
{
    QDW_CHECK(ops && etas && psis && p && work && infos, QDW_EINVAL,
              "sap_gcr_solve_batched: null argument");
    QDW_CHECK(n >= 1, QDW_EINVAL, "sap_gcr_solve_batched: need n >= 1");
    int rc = check_params(p);
    if (rc) return rc;
    qdw_batch* b = nullptr;
    if ((rc = qdw_batch_create(ops, n, p, 1, work, work_bytes, &b))) return rc;
    if (graph_ms) *graph_ms = b->capture_ms;
    rc = qdw_batch_solve(b, etas, psis, infos, nullptr, stream);
    qdw_batch_destroy(b);
    return rc;
}
