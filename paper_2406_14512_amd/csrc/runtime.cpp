// Host runtime behind the C ABI of include/ffpic.h: descriptor validation,
// FP64 geometry tables, initial fields, device allocations, the step
// sequence, particle load/export, diagnostics and checkpoints.  No C++
// exception crosses the ABI: every entry point catches and maps to a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "ffpic_internal.h"

namespace ffpic {
void field_step64(ffpic_ctx *c);
void field_step32(ffpic_ctx *c);
void psi_mask64(ffpic_ctx *c);
void psi_mask32(ffpic_ctx *c);
void push64(ffpic_ctx *c, int s);
void push32(ffpic_ctx *c, int s);

template <typename R>
static Geo<R> make_geo(const ffpic_ctx *c, R *const *t) {
    Geo<R> g;
    g.nr = c->nr; g.nth = c->nth; g.ld = c->ld;
    g.dt = (R)c->dt; g.dth = (R)c->dth;
    g.rn = t[T_RN]; g.rh = t[T_RH]; g.rn2 = t[T_RN2]; g.rh2 = t[T_RH2];
    g.drn = t[T_DRN]; g.drh = t[T_DRH]; g.dr2n = t[T_DR2N]; g.dr2h = t[T_DR2H];
    g.dr3h = t[T_DR3H]; g.dr3n = t[T_DR3N]; g.lamn = t[T_LAMN]; g.lamh = t[T_LAMH];
    g.sn = t[T_SN]; g.cn = t[T_CN]; g.sh = t[T_SH]; g.dcn = t[T_DCN]; g.dcd = t[T_DCD];
    g.dthd = t[T_DTHD];
    return g;
}
template <>
Geo<double> geo<double>(const ffpic_ctx *c) { return make_geo<double>(c, c->dtab64); }
template <>
Geo<float> geo<float>(const ffpic_ctx *c) { return make_geo<float>(c, (float *const *)c->dtab); }

void psi_mask(ffpic_ctx *c) { c->fp64 ? psi_mask64(c) : psi_mask32(c); }
void field_step(ffpic_ctx *c) { c->fp64 ? field_step64(c) : field_step32(c); }
void push_species(ffpic_ctx *c, int s) { c->fp64 ? push64(c, s) : push32(c, s); }
}  // namespace ffpic

using namespace ffpic;

namespace {

struct Fail {
    int code;
    std::string msg;
};

#define HCHK(x)                                                                       \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess)                                                         \
            throw Fail{FFPIC_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)};   \
    } while (0)

template <typename F>
int guarded(ffpic_ctx *c, F &&f) {
    try {
        f();
        return FFPIC_OK;
    } catch (const Fail &e) {
        if (c) c->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->last_error = "host allocation failed";
        return FFPIC_ENOMEM;
    } catch (const std::exception &e) {
        if (c) c->last_error = e.what();
        return FFPIC_EHIP;
    }
}

void *dmalloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Fail{FFPIC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    return p;
}

std::string validate(const ffpic_desc *d) {
    if (!d) return "descriptor is NULL";
    if (d->nr < 2 || d->nth < 2 || d->nr > 65535 || d->nth > 65535)
        return "nr and nth must lie in [2, 65535]";
    // the kernels address field arrays with 32-bit byte offsets
    if ((int64_t)(d->nr + 1) * (d->nth + 1) > (int64_t(1) << 29))
        return "grid too large: (nr+1)*(nth+1) must not exceed 2^29";
    if (!(d->rmin > 0) || !(d->rmax > d->rmin) || !std::isfinite(d->rmax))
        return "need 0 < rmin < rmax";
    if (!(d->r_abs > d->rmin) || !(d->r_abs <= d->rmax)) return "need rmin < r_abs <= rmax";
    if (!(d->cfl > 0) || !(d->cfl <= 1)) return "cfl must lie in (0, 1]";
    if (!(d->r_lc > 0) || !std::isfinite(d->r_lc)) return "r_lc must be positive";
    if (!std::isfinite(d->mu) || !std::isfinite(d->omega_b) || !std::isfinite(d->rr_coef))
        return "mu, omega_b and rr_coef must be finite";
    for (int k = 0; k < 4; k++)
        if (std::isnan(d->psi_thr[k])) return "psi thresholds must not be NaN";
    for (int k = 0; k < 3; k++)
        if (!(d->psi_thr[k] <= d->psi_thr[k + 1])) return "psi thresholds must be non-decreasing";
    if (d->precision != FFPIC_FP64 && d->precision != FFPIC_FP32_MIXED) return "bad precision";
    if (d->init < FFPIC_INIT_ZERO || d->init > FFPIC_INIT_OPEN_DIPOLE) return "bad init";
    if (d->sort_interval < 0) return "sort_interval must be >= 0 (0 = tuned)";
    if (d->nspec < 0 || d->nspec > FFPIC_MAX_SPECIES) return "nspec out of range";
    for (int s = 0; s < d->nspec; s++) {
        if (d->capacity[s] < 0 || d->capacity[s] > (int64_t(1) << 30))
            return "capacity out of range [0, 2^30]";
        if (!std::isfinite(d->qm[s]) || d->qm[s] == 0.0) return "qm must be finite and non-zero";
        if (!std::isfinite(d->weight[s]) || d->weight[s] < 0) return "weight must be >= 0";
    }
    if (!std::isfinite(d->inject_kappa) || d->inject_kappa < 0) return "inject_kappa must be >= 0";
    if (d->inject_kappa > 0 && d->nspec > 0 && !(d->weight[0] > 0))
        return "injection needs weight[0] > 0";
    if (d->rr_ramp_n < 0 || d->rr_ramp_n > 4) return "rr_ramp_n must lie in [0, 4]";
    for (int k = 0; k < d->rr_ramp_n; k++) {
        if (!std::isfinite(d->rr_ramp_t[k]) || !std::isfinite(d->rr_ramp_f[k]) ||
            d->rr_ramp_f[k] < 0)
            return "ramp knots must be finite with factors >= 0";
        if (k > 0 && !(d->rr_ramp_t[k] >= d->rr_ramp_t[k - 1]))
            return "ramp knot times must be non-decreasing";
    }
    if (!(d->shell_r >= 0) || !std::isfinite(d->shell_r)) return "shell_r must be >= 0";
    if (!(d->gj_extract >= 0) || !std::isfinite(d->gj_extract)) return "gj_extract must be >= 0";
    if (d->gj_extract > 0) {
        for (int k = 0; k < 2; k++)
            if (d->gj_species[k] < 0 || d->gj_species[k] >= d->nspec)
                return "gj_species out of range";
        if (d->gj_species[0] == d->gj_species[1]) return "gj_species must differ";
        if (!(d->weight[d->gj_species[0]] + d->weight[d->gj_species[1]] > 0))
            return "extraction needs positive weights";
    }
    if (!(d->gamma_th >= 0) || !std::isfinite(d->gamma_th)) return "gamma_th must be >= 0";
    if (d->gamma_th > 0) {
        if (!(d->gamma_s >= 1) || !(d->gamma_s < d->gamma_th))
            return "need 1 <= gamma_s < gamma_th";
        for (int k = 0; k < 2; k++)
            if (d->pair_species[k] < 0 || d->pair_species[k] >= d->nspec)
                return "pair_species out of range";
        if (d->pair_species[0] == d->pair_species[1]) return "pair_species must differ";
    }
    return "";
}

void build_tables(ffpic_ctx *c);

// grid sizes, spacings, time step and the geometry tables of a descriptor
// (host only; no device call)
void setup_geometry(ffpic_ctx *c, const ffpic_desc *d) {
    c->d = *d;
    c->nr = d->nr; c->nth = d->nth; c->ld = d->nth + 1;
    c->nn = (size_t)(d->nr + 1) * (size_t)(d->nth + 1);
    c->fp64 = d->precision == FFPIC_FP64;
    c->rsz = c->fp64 ? sizeof(double) : sizeof(float);
    c->dlog = std::log(d->rmax / d->rmin) / d->nr;
    c->dth = kPi / d->nth;
    c->omega = 1.0 / d->r_lc;
    {   // CFL number times the 2-D Courant limit of the innermost cell
        double r0 = d->rmin, r1 = d->rmin * std::exp(c->dlog);
        double drr = r1 - r0, drt = r0 * c->dth;
        c->dt = d->cfl / std::sqrt(1.0 / (drr * drr) + 1.0 / (drt * drt));
    }
    build_tables(c);
}

// geometry tables (FP64, on the host)
void build_tables(ffpic_ctx *c) {
    const int nr = c->nr, nth = c->nth;
    const double rmin = c->d.rmin;
    auto &T = c->tab;
    for (auto &t : T) t.clear();
    T[T_RN].resize(nr + 1); T[T_RH].resize(nr); T[T_RN2].resize(nr + 1); T[T_RH2].resize(nr);
    T[T_DRN].resize(nr); T[T_DRH].resize(nr + 1); T[T_DR2N].resize(nr); T[T_DR2H].resize(nr + 1);
    T[T_DR3H].resize(nr + 1); T[T_DR3N].resize(nr); T[T_LAMN].resize(nr + 1); T[T_LAMH].resize(nr);
    T[T_SN].resize(nth + 1); T[T_CN].resize(nth + 1); T[T_SH].resize(nth); T[T_DCN].resize(nth);
    T[T_DCD].resize(nth + 1); T[T_DTHD].resize(nth + 1); T[T_THN].resize(nth + 1);
    auto &rn = T[T_RN], &rh = T[T_RH];
    for (int i = 0; i <= nr; i++) rn[i] = rmin * std::exp(i * c->dlog);
    for (int i = 0; i < nr; i++) rh[i] = rmin * std::exp((i + 0.5) * c->dlog);
    for (int i = 0; i <= nr; i++) T[T_RN2][i] = rn[i] * rn[i];
    for (int i = 0; i < nr; i++) T[T_RH2][i] = rh[i] * rh[i];
    for (int i = 0; i < nr; i++) T[T_DRN][i] = rn[i + 1] - rn[i];
    for (int i = 0; i <= nr; i++) T[T_DRH][i] = (i >= 1 && i < nr) ? rh[i] - rh[i - 1] : 0.0;
    for (int i = 0; i < nr; i++) T[T_DR2N][i] = (rn[i + 1] * rn[i + 1] - rn[i] * rn[i]) * 0.5;
    for (int i = 0; i <= nr; i++) {
        double lo = i == 0 ? rn[0] : rh[i - 1];
        double hi = i == nr ? rn[nr] : rh[i];
        T[T_DR2H][i] = (hi * hi - lo * lo) * 0.5;
        T[T_DR3H][i] = (hi * hi * hi - lo * lo * lo) / 3.0;
    }
    for (int i = 0; i < nr; i++)
        T[T_DR3N][i] = (rn[i + 1] * rn[i + 1] * rn[i + 1] - rn[i] * rn[i] * rn[i]) / 3.0;
    // absorbing layer (Sect. 4): lambda = exp(-sigma0 dt x^3) beyond r_abs,
    // x = (r - r_abs) / (rmax - r_abs), sigma0 = 40 / (rmax - r_abs)
    auto absorb = [&](double r) {
        if (!(r > c->d.r_abs)) return 1.0;
        double L = c->d.rmax - c->d.r_abs;
        double x = (r - c->d.r_abs) / L;
        return std::exp(-(40.0 / L) * c->dt * x * x * x);
    };
    for (int i = 0; i <= nr; i++) T[T_LAMN][i] = absorb(rn[i]);
    for (int i = 0; i < nr; i++) T[T_LAMH][i] = absorb(rh[i]);
    std::vector<double> ch(nth);
    for (int j = 0; j <= nth; j++) {
        T[T_THN][j] = j * c->dth;
        T[T_SN][j] = std::sin(T[T_THN][j]);
        T[T_CN][j] = std::cos(T[T_THN][j]);
    }
    T[T_SN][0] = 0.0; T[T_CN][0] = 1.0; T[T_SN][nth] = 0.0; T[T_CN][nth] = -1.0;
    for (int j = 0; j < nth; j++) {
        T[T_SH][j] = std::sin((j + 0.5) * c->dth);
        ch[j] = std::cos((j + 0.5) * c->dth);
    }
    for (int j = 0; j < nth; j++) T[T_DCN][j] = T[T_CN][j] - T[T_CN][j + 1];
    for (int j = 0; j <= nth; j++) {
        double lo = j == 0 ? 1.0 : ch[j - 1];
        double hi = j == nth ? -1.0 : ch[j];
        T[T_DCD][j] = lo - hi;
        T[T_DTHD][j] = (j == 0 || j == nth) ? 0.5 * c->dth : c->dth;
    }
}

double psi_init(const ffpic_ctx *c, int i, int j) {
    double r = c->tab[T_RN][i], st = c->tab[T_SN][j], ct = c->tab[T_CN][j], mu = c->d.mu;
    switch (c->d.init) {
    case FFPIC_INIT_DIPOLE:
        return mu * st * st / r;
    case FFPIC_INIT_MONOPOLE:
    case FFPIC_INIT_MICHEL:
        return mu * (1.0 - ct);
    case FFPIC_INIT_OPEN_DIPOLE: {
        double cs = r < c->d.r_lc ? std::sqrt(1.0 - r / c->d.r_lc) : 0.0;
        if (std::fabs(ct) < cs) return mu * st * st / r;
        return mu / c->d.r_lc * (1.0 - std::fabs(ct)) / (1.0 - cs);
    }
    default:
        return 0.0;
    }
}

// initial fields from nodal Psi differences (exactly divergence-free B) and
// the corotation field E = -Omega grad Psi in edge form
void init_fields_host(const ffpic_ctx *c, std::vector<double> F[6]) {
    const int nr = c->nr, nth = c->nth, ld = c->ld;
    for (int k = 0; k < 6; k++) F[k].assign(c->nn, 0.0);
    if (c->d.init == FFPIC_INIT_ZERO) return;
    std::vector<double> ps(c->nn);
    auto PS = [&](int i, int j) -> double & { return ps[(size_t)i * ld + j]; };
    auto at = [&](int k, int i, int j) -> double & { return F[k][(size_t)i * ld + j]; };
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j <= nth; j++) PS(i, j) = psi_init(c, i, j);
    const auto &T = c->tab;
    double om = c->omega;
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j < nth; j++) {
            at(3, i, j) = (PS(i, j + 1) - PS(i, j)) / (T[T_RN2][i] * T[T_DCN][j]);
            at(1, i, j) = i == nr ? 0.0 : -om * (PS(i, j + 1) - PS(i, j)) / (T[T_RN][i] * c->dth);
        }
    for (int i = 0; i < nr; i++)
        for (int j = 0; j <= nth; j++) {
            if (j > 0 && j < nth)
                at(4, i, j) = -(PS(i + 1, j) - PS(i, j)) / (T[T_SN][j] * T[T_DR2N][i]);
            at(0, i, j) = -om * (PS(i + 1, j) - PS(i, j)) / T[T_DRN][i];
        }
    if (c->d.init == FFPIC_INIT_MICHEL)
        for (int i = 0; i < nr; i++)
            for (int j = 0; j < nth; j++)
                at(5, i, j) = -om * (PS(i, j + 1) - PS(i, j)) / (T[T_RH][i] * c->dth);
}

void upload_field(ffpic_ctx *c, void *dst, const std::vector<double> &h) {
    if (c->fp64) {
        HCHK(hipMemcpyAsync(dst, h.data(), c->nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
    } else {
        std::vector<float> f(h.begin(), h.end());
        HCHK(hipMemcpyAsync(dst, f.data(), c->nn * sizeof(float), hipMemcpyHostToDevice, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
    }
}

// FP32 mode: rates of the FP64 background fields under the discrete
// operators of the field step, evaluated in FP64 (see fields_fused.h):
// Faraday rate -curl E0 at B positions, Ampere rate curl B0 at the E
// positions the step updates, and rho0 = div E0 / 4 pi at nodes.
void upload_background(ffpic_ctx *c) {
    const int nr = c->nr, nth = c->nth, ld = c->ld;
    const auto &T = c->tab;
    const auto &E0 = c->hE0, &B0 = c->hB0;
    std::vector<double> rB[3], rE[3], rho(c->nn, 0.0);
    for (int k = 0; k < 3; k++) { rB[k].assign(c->nn, 0.0); rE[k].assign(c->nn, 0.0); }
    auto at = [&](const std::vector<double> &a, int i, int j) { return a[(size_t)i * ld + j]; };
    auto set = [&](std::vector<double> &a, int i, int j, double v) { a[(size_t)i * ld + j] = v; };
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j <= nth; j++) {
            if (j < nth) {
                double circ = T[T_RN][i] * (T[T_SN][j + 1] * at(E0[2], i, j + 1) - T[T_SN][j] * at(E0[2], i, j));
                set(rB[0], i, j, -circ / (T[T_RN2][i] * T[T_DCN][j]));
            }
            if (i < nr) {
                if (j > 0 && j < nth) {
                    double circ = T[T_SN][j] * (T[T_RN][i + 1] * at(E0[2], i + 1, j) - T[T_RN][i] * at(E0[2], i, j));
                    set(rB[1], i, j, circ / (T[T_SN][j] * T[T_DR2N][i]));
                }
                if (j < nth) {
                    double circ = c->dth * (T[T_RN][i + 1] * at(E0[1], i + 1, j) - T[T_RN][i] * at(E0[1], i, j)) -
                                  T[T_DRN][i] * (at(E0[0], i, j + 1) - at(E0[0], i, j));
                    set(rB[2], i, j, -circ / (c->dth * T[T_DR2N][i]));
                }
                double A = T[T_RH2][i] * T[T_DCD][j];
                double circ = (j < nth ? T[T_RH][i] * T[T_SH][j] * at(B0[2], i, j) : 0.0) -
                              (j > 0 ? T[T_RH][i] * T[T_SH][j - 1] * at(B0[2], i, j - 1) : 0.0);
                set(rE[0], i, j, circ / A);
            }
            if (i >= 1 && i < nr) {
                if (j < nth) {
                    double A = T[T_SH][j] * T[T_DR2H][i];
                    double circ = -(T[T_RH][i] * T[T_SH][j] * at(B0[2], i, j) -
                                    T[T_RH][i - 1] * T[T_SH][j] * at(B0[2], i - 1, j));
                    set(rE[1], i, j, circ / A);
                }
                if (j >= 1 && j < nth) {
                    double A = T[T_DTHD][j] * T[T_DR2H][i];
                    double circ = c->dth * (T[T_RH][i] * at(B0[1], i, j) - T[T_RH][i - 1] * at(B0[1], i - 1, j)) -
                                  T[T_DRH][i] * (at(B0[0], i, j) - at(B0[0], i, j - 1));
                    set(rE[2], i, j, circ / A);
                }
            }
        }
    auto dive = [&](int i, int j) {
        double flux = T[T_RH2][i] * T[T_DCD][j] * at(E0[0], i, j) -
                      T[T_RH2][i - 1] * T[T_DCD][j] * at(E0[0], i - 1, j);
        if (j < nth) flux += T[T_SH][j] * T[T_DR2H][i] * at(E0[1], i, j);
        if (j > 0) flux -= T[T_SH][j - 1] * T[T_DR2H][i] * at(E0[1], i, j - 1);
        return flux / (T[T_DR3H][i] * T[T_DCD][j]);
    };
    for (int i = 0; i < nr; i++)
        for (int j = 0; j <= nth; j++) set(rho, i, j, dive(i == 0 ? 1 : i, j) / (4.0 * kPi));
    // A rate that is identically zero (curl B0 of a field without B_phi) is
    // not read by the field step.  Nor is a Faraday rate -curl E0 that is
    // FP64 rounding of a curl-free background (the corotation field
    // E0 = -Omega grad Psi of every initial state): below 1e-9 of
    // max |E0| / dr_0 it changes no FP32 perturbation.
    double emax = 0.0;
    for (int k = 0; k < 3; k++)
        for (double v : E0[k]) emax = std::max(emax, std::fabs(v));
    const double rb_floor = 1e-9 * emax / T[T_DRN][0];
    for (int k = 0; k < 3; k++) {
        c->rE0_zero[k] = std::all_of(rE[k].begin(), rE[k].end(), [](double v) { return v == 0.0; });
        c->rB0_zero[k] = std::all_of(rB[k].begin(), rB[k].end(),
                                     [&](double v) { return std::fabs(v) <= rb_floor; });
    }
    auto up = [&](void *dst, const std::vector<double> &h) {
        std::vector<float> f(h.begin(), h.end());
        HCHK(hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    };
    for (int k = 0; k < 3; k++) {
        up(c->rB0[k], rB[k]);
        up(c->rE0[k], rE[k]);
        up(c->E0[k], E0[k]);
    }
    for (int k = 0; k < 2; k++) {
        HCHK(hipMemcpy(c->E0d[k], E0[k].data(), c->nn * sizeof(double), hipMemcpyHostToDevice));
        HCHK(hipMemcpy(c->B0d[k], B0[k].data(), c->nn * sizeof(double), hipMemcpyHostToDevice));
    }
    up(c->rho0, rho);
}

// one device allocation for the three components of a field, cstride
// elements apart (the pointers of the components go to p[0..2])
void alloc3(ffpic_ctx *c, void **p, bool zero) {
    const size_t cs = c->cstride * c->rsz;
    char *b = (char *)dmalloc(3 * cs);
    if (zero) HCHK(hipMemset(b, 0, 3 * cs));
    for (int k = 0; k < 3; k++) p[k] = b + k * cs;
}

void destroy_graphs(ffpic_ctx *c);

void free_all(ffpic_ctx *c) {
    destroy_graphs(c);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->gfork) (void)hipEventDestroy(c->gfork);
    if (c->gjoin) (void)hipEventDestroy(c->gjoin);
    c->gstream = nullptr;
    c->gfork = c->gjoin = nullptr;
    auto F = [](void *p) { if (p) (void)hipFree(p); };
    // three-component fields: one allocation each, at component 0
    F(c->dE[0]); F(c->dB[0]); F(c->E0[0]); F(c->rE0[0]); F(c->rB0[0]);
    for (int k = 0; k < 2; k++) { F(c->E0d[k]); F(c->B0d[k]); }
    F(c->rho0);
    for (int t = 0; t < T_NTAB; t++) {
        if (c->dtab[t] != (void *)c->dtab64[t]) F(c->dtab[t]);
        F(c->dtab64[t]);
    }
    F(c->E[0]); F(c->B[0]); F(c->B0[0]); F(c->J[0]); F(c->Jalt[0]);
    F(c->stAlt[0]); F(c->stAlt[3]);
    F(c->fz_rowc); F(c->fz_colc);
    F(c->psi); F(c->f); F(c->kill);
    for (int s = 0; s < FFPIC_MAX_SPECIES; s++)
        for (int a = 0; a < 6; a++) { F(c->sp[s].cur[a]); F(c->sp[s].alt[a]); }
    for (int k = 0; k < 2; k++) { F(c->keys[k]); F(c->vals[k]); }
    for (int s = 0; s < FFPIC_MAX_SPECIES; s++)
        for (int k = 0; k < 2; k++) F(c->soff[s][k]);
    for (int s = 0; s < FFPIC_MAX_SPECIES; s++) {
        F(c->sort_smask[s]); F(c->sort_mmask[s]); F(c->sort_wsm[s]); F(c->sort_tc[s]);
        F(c->sort_ts[s]); F(c->sort_gs[s]); F(c->sort_tot[s]); F(c->sort_mst[s]);
        F(c->sort_dest[s]);
    }
    F(c->sort_aux); F(c->sort_kcnt); F(c->sort_cbuf);
    F(c->rs_hist); F(c->rs_dtot); F(c->rs_n); F(c->scan_part);
    for (int s = 0; s < FFPIC_MAX_SPECIES; s++) F(c->perm[s]);
    F(c->inj_rate); F(c->inj_cnt); F(c->inj_off); F(c->nsorted);
    F(c->gj_target); F(c->gj_have); F(c->pair_cnt); F(c->pair_off);
    F(c->spec_tab); F(c->spec_edge); F(c->spec_nu);
    F(c->nslots); F(c->nalive); F(c->removed); F(c->err); F(c->red);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->evpool) (void)hipEventDestroy(e);
    c->evpool.clear();
}

// Tables of the surface sources from the surface B_r (FP64, the same
// operation order as the oracle's definitions), V the volume of surface cell
// (0, j) per radian of azimuth and |rho_GJ| = Omega |B_r| / 2 pi:
//   pairs injected per step: kappa_inj |rho_GJ| / q * V * dt / dr0;
//   charge kept by the extraction: gj_extract |rho_GJ| V.
void surface_tables(ffpic_ctx *c, const double *br_surface) {
#pragma clang fp contract(off)
    const bool inj = c->d.inject_kappa > 0.0 && c->d.nspec > 0;
    const bool ext = c->d.gj_extract > 0.0;
    if (!inj && !ext) return;
    const int nth = c->nth;
    const std::vector<double> &rn = c->tab[T_RN], &cn = c->tab[T_CN];
    std::vector<double> rate(nth), target(nth);
    double ibound = 0.0, ebound = 0.0;   // most particles a step adds (sums of ceilings)
    const double wpair = ext ? c->d.weight[c->d.gj_species[0]] + c->d.weight[c->d.gj_species[1]]
                             : 1.0;
    for (int j = 0; j < nth; j++) {
        const double br = std::fabs(br_surface[j]);
        const double vol = (rn[1] * rn[1] * rn[1] - rn[0] * rn[0] * rn[0]) / 3.0 * (cn[j] - cn[j + 1]);
        if (inj) {
            const double q = c->d.weight[0];
            rate[j] = c->d.inject_kappa * (c->omega * br / (2.0 * kPi)) / q * vol *
                      (c->dt / (rn[1] - rn[0]));
            ibound += std::ceil(rate[j]);
        }
        if (ext) {
            target[j] = c->d.gj_extract * (c->omega * br / (2.0 * kPi)) * vol;
            ebound += std::ceil(target[j] / wpair);
        }
    }
    // per-cell counts and their scan are int32: the most a step can add must
    // stay far below 2^31
    if (!(ibound <= 1073741824.0) || !(ebound <= 1073741824.0))
        throw Fail{FFPIC_EINVAL, "a surface source would add more than 2^30 particles in one "
                                 "step: raise the weights"};
    if (!c->inj_cnt) {
        c->inj_cnt = (int32_t *)dmalloc((size_t)(nth + 1) * sizeof(int32_t));
        c->inj_off = (int32_t *)dmalloc((size_t)(nth + 1) * sizeof(int32_t));
    }
    if (inj) {
        if (!c->inj_rate) c->inj_rate = (double *)dmalloc((size_t)nth * sizeof(double));
        HCHK(hipMemcpy(c->inj_rate, rate.data(), (size_t)nth * sizeof(double), hipMemcpyHostToDevice));
        c->inj_bound = (int64_t)ibound;
    }
    if (ext) {
        if (!c->gj_target) {
            c->gj_target = (double *)dmalloc((size_t)nth * sizeof(double));
            c->gj_have = (int32_t *)dmalloc((size_t)c->d.nspec * nth * sizeof(int32_t));
        }
        HCHK(hipMemcpy(c->gj_target, target.data(), (size_t)nth * sizeof(double),
                       hipMemcpyHostToDevice));
        c->gj_bound = (int64_t)ebound;
    }
}

// radiation-reaction ramp at t = step * dt: piecewise linear through the
// knots, flat outside them (the same operation order as the oracle's)
double rr_factor_at(const ffpic_desc &d, double t) {
#pragma clang fp contract(off)
    const int n = d.rr_ramp_n;
    if (n <= 0) return 1.0;
    if (t <= d.rr_ramp_t[0]) return d.rr_ramp_f[0];
    for (int k = 1; k < n; k++) {
        if (t < d.rr_ramp_t[k]) {
            const double t0 = d.rr_ramp_t[k - 1], t1 = d.rr_ramp_t[k];
            const double x = (t - t0) / (t1 - t0);
            return d.rr_ramp_f[k - 1] + x * (d.rr_ramp_f[k] - d.rr_ramp_f[k - 1]);
        }
    }
    return d.rr_ramp_f[n - 1];
}

void check_ctx(ffpic_ctx *c) {
    if (!c) throw Fail{FFPIC_EINVAL, "context is NULL"};
}

int read_err(ffpic_ctx *c) {
    uint32_t e = 0;
    HCHK(hipMemcpyAsync(&e, c->err, sizeof(e), hipMemcpyDeviceToHost, c->stream));
    HCHK(hipStreamSynchronize(c->stream));
    if (e) {
        std::string m = "device error word 0x" + std::to_string(e) + ":";
        if (e & FFPIC_ERR_NONFINITE) m += " non-finite momentum;";
        if (e & FFPIC_ERR_CFL) m += " particle crossed more than one cell in a step;";
        if (e & FFPIC_ERR_CAPACITY) m += " injection exceeded a species' capacity;";
        const bool numeric = (e & (FFPIC_ERR_NONFINITE | FFPIC_ERR_CFL)) != 0;
        throw Fail{numeric ? FFPIC_ENUMERIC : FFPIC_ECAPACITY, m};
    }
    return 0;
}

void one_step(ffpic_ctx *c, uint32_t ph, bool count_step, int tslot) {
    auto mark = [&](int k) {
        if (c->timing && tslot >= 0) HCHK(hipEventRecord(c->evpool[5 * tslot + k], c->stream));
    };
    mark(0);
    if (ph & FFPIC_PHASE_MASK) psi_mask(c);
    mark(1);
    // FP32: when this step pushes and nothing is appended between the sort
    // and the push, the push writes its particles in the sorted order (one
    // pass over the state instead of two)
    const bool defer = (ph & FFPIC_PHASE_PUSH) && !c->fp64 &&
                       !((ph & FFPIC_PHASE_INJECT) && c->d.inject_kappa > 0.0) &&
                       !((ph & FFPIC_PHASE_EXTRACT) && c->d.gj_extract > 0.0);
    for (int s = 0; s < c->d.nspec; s++) {
        if (ph & FFPIC_PHASE_SORT) sort_species(c, s, defer);
        else if (ph & FFPIC_PHASE_KILL) kill_species(c, s);
    }
    const bool sources = (c->d.inject_kappa > 0.0 || c->d.gj_extract > 0.0 ||
                          c->d.gamma_th > 0.0) && c->d.nspec > 0;
    if (sources) {
        // the sources add particles that only the device counts: every
        // launch covers all slots of a species (each kernel stops at the
        // device count), so no count is read back during the step
        for (int s = 0; s < c->d.nspec; s++) c->sp[s].nub = c->sp[s].cap;
    }
    if (ph & FFPIC_PHASE_INJECT) inject_pairs(c);
    if (ph & FFPIC_PHASE_EXTRACT) extract_gj(c);
    mark(2);
    if (ph & FFPIC_PHASE_PUSH)
        for (int s = 0; s < c->d.nspec; s++) push_species(c, s);
    if (ph & FFPIC_PHASE_PAIRS) create_pairs(c);
    mark(3);
    if (ph & FFPIC_PHASE_FIELDS) field_step(c);
    mark(4);
    if (count_step) c->step++;
}

// phases of the step about to be taken
uint32_t step_phases(const ffpic_ctx *c) {
    uint32_t ph = FFPIC_PHASE_MASK | FFPIC_PHASE_KILL | FFPIC_PHASE_INJECT | FFPIC_PHASE_EXTRACT |
                  FFPIC_PHASE_PUSH | FFPIC_PHASE_PAIRS | FFPIC_PHASE_FIELDS;
    if (c->step % c->d.sort_interval == 0) ph |= FFPIC_PHASE_SORT;
    // the push removes particles of force-free cells itself
    if (!(ph & FFPIC_PHASE_SORT)) ph &= ~FFPIC_PHASE_KILL;
    return ph;
}

CycleState cycle_state(const ffpic_ctx *c) {
    CycleState st;
    std::memset(&st, 0, sizeof(st));   // compared bytewise, padding included
    for (int s = 0; s < FFPIC_MAX_SPECIES; s++) {
        for (int a = 0; a < 6; a++) {
            st.cur[s][a] = c->sp[s].cur[a];
            st.alt[s][a] = c->sp[s].alt[a];
        }
        st.nub[s] = c->sp[s].nub;
        st.sort_cur[s] = c->sort_cur[s];
        st.sort_valid[s] = c->sort_valid[s];
        st.perm_valid[s] = c->perm_valid[s];
    }
    for (int k = 0; k < 3; k++) {
        st.E[k] = c->E[k];
        st.B[k] = c->B[k];
        st.J[k] = c->J[k];
        st.dE[k] = c->dE[k];
        st.dB[k] = c->dB[k];
        st.Jalt[k] = c->Jalt[k];
    }
    for (int k = 0; k < 6; k++) st.stAlt[k] = c->stAlt[k];
    st.fused_rows = c->fused_rows;
    st.push_ppt = c->push_ppt;
    st.record_perm = c->record_perm;
    st.incremental_sort = c->incremental_sort;
    return st;
}

void set_cycle_state(ffpic_ctx *c, const CycleState &st) {
    for (int s = 0; s < FFPIC_MAX_SPECIES; s++) {
        for (int a = 0; a < 6; a++) {
            c->sp[s].cur[a] = st.cur[s][a];
            c->sp[s].alt[a] = st.alt[s][a];
        }
        c->sp[s].nub = st.nub[s];
        c->sort_cur[s] = st.sort_cur[s];
        c->sort_valid[s] = st.sort_valid[s];
        c->perm_valid[s] = st.perm_valid[s];
    }
    for (int k = 0; k < 3; k++) {
        c->E[k] = st.E[k];
        c->B[k] = st.B[k];
        c->J[k] = st.J[k];
        c->dE[k] = st.dE[k];
        c->dB[k] = st.dB[k];
        c->Jalt[k] = st.Jalt[k];
    }
    for (int k = 0; k < 6; k++) c->stAlt[k] = st.stAlt[k];
}

// A sort cycle can be replayed from a graph when no kernel argument
// depends on the step number (the surface sources draw from a counter-based
// generator keyed by the step; a radiation-reaction ramp changes the push's
// coefficient every step), and every species with particles has had its
// first (full) sort.
bool cycle_graphable(const ffpic_ctx *c) {
    if (!c->use_graph || c->timing) return false;
    if (c->d.inject_kappa > 0.0 || c->d.gj_extract > 0.0 || c->d.rr_ramp_n > 0) return false;
    for (int s = 0; s < c->d.nspec; s++)
        if (c->sp[s].nub > 0 && !c->sort_valid[s]) return false;
    return true;
}

constexpr size_t kMaxGraphs = 4;

void destroy_graphs(ffpic_ctx *c) {
    if (!c->graphs.empty() && c->gstream) (void)hipStreamSynchronize(c->gstream);
    for (auto &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

void launch_graph(ffpic_ctx *c, hipGraphExec_t exec) {
    // the graph runs on the capture stream, ordered after the work already
    // on the context's stream and before the work that follows it there
    HCHK(hipEventRecord(c->gfork, c->stream));
    HCHK(hipStreamWaitEvent(c->gstream, c->gfork, 0));
    HCHK(hipGraphLaunch(exec, c->gstream));
    HCHK(hipEventRecord(c->gjoin, c->gstream));
    HCHK(hipStreamWaitEvent(c->stream, c->gjoin, 0));
    c->graph_launches++;
}

// k steps from a sort step, as one graph: replayed if one was captured from
// the same host state, else captured (the host bookkeeping of the steps runs
// while the kernels are recorded), instantiated and kept
void run_cycle_graph(ffpic_ctx *c, int k) {
    const CycleState pre = cycle_state(c);
    for (auto &g : c->graphs) {
        if (g.steps == k && std::memcmp(&g.pre, &pre, sizeof(pre)) == 0) {
            launch_graph(c, g.exec);
            set_cycle_state(c, g.post);
            c->step += k;
            return;
        }
    }
    if (!c->gstream) {
        HCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HCHK(hipEventCreateWithFlags(&c->gfork, hipEventDisableTiming));
        HCHK(hipEventCreateWithFlags(&c->gjoin, hipEventDisableTiming));
    }
    const int64_t step0 = c->step;
    hipStream_t saved = c->stream;
    c->stream = c->gstream;
    hipGraph_t graph = nullptr;
    HCHK(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
    try {
        for (int i = 0; i < k; i++) one_step(c, step_phases(c), true, -1);
    } catch (...) {
        (void)hipStreamEndCapture(c->gstream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        c->stream = saved;
        set_cycle_state(c, pre);
        c->step = step0;
        throw;
    }
    c->stream = saved;
    HCHK(hipStreamEndCapture(c->gstream, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        set_cycle_state(c, pre);
        c->step = step0;
        throw Fail{FFPIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    }
    if (c->graphs.size() >= kMaxGraphs) destroy_graphs(c);
    CycleGraph g;
    g.steps = k;
    g.pre = pre;
    g.post = cycle_state(c);
    g.exec = exec;
    c->graphs.push_back(g);
    c->graph_builds++;
    launch_graph(c, exec);
}

}  // namespace

namespace ffpic {

static double host_max(ffpic_ctx *c, const double *part) {
    double h[1024];
    const int n = diag_partials();
    if (n > 1024) throw Fail{FFPIC_EINVAL, "too many partials"};
    HCHK(hipMemcpyAsync(h, part, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HCHK(hipStreamSynchronize(c->stream));
    double m = 0.0;
    for (int k = 0; k < n; k++) m = h[k] > m ? h[k] : m;
    return m;
}

void run_diagnostics(ffpic_ctx *c, uint32_t what, ffpic_diag *out, double *L, const DiagBufs &b) {
    std::memset(out, 0, sizeof(*out));
    out->step = c->step;
    HCHK(hipStreamSynchronize(c->stream));
    unsigned long long rem[FFPIC_MAX_SPECIES * 4];
    HCHK(hipMemcpy(rem, c->removed, sizeof(rem), hipMemcpyDeviceToHost));
    HCHK(hipMemcpy(&out->error_word, c->err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    for (int s = 0; s < c->d.nspec; s++)
        for (int k = 0; k < 4; k++) out->removed[s][k] = (int64_t)rem[4 * s + k];
    if (what & FFPIC_DIAG_MOMENTS) {
        for (int s = 0; s < c->d.nspec; s++) {
            moments(c, s, b.part, b.out);
            double h[5];
            HCHK(hipMemcpyAsync(h, b.out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
            HCHK(hipStreamSynchronize(c->stream));
            out->alive[s] = (int64_t)h[0];
            out->sum_gamma[s] = h[1];
            for (int k = 0; k < 3; k++) out->sum_u[s][k] = h[2 + k];
        }
    }
    if (what & FFPIC_DIAG_ENERGY) {
        energies(c, b.part, b.out);
        double h[2];
        HCHK(hipMemcpyAsync(h, b.out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        out->energy_e = h[0];
        out->energy_b = h[1];
    }
    if (what & FFPIC_DIAG_RESIDUALS) {
        gauss(c, b.qn, nullptr, b.part);
        out->gauss_max = host_max(c, b.part);
        divb(c, nullptr, b.part);
        out->divb_max = host_max(c, b.part);
    }
    if ((what & FFPIC_DIAG_POYNTING) && L) {
        poynting(c, b.L);
        HCHK(hipMemcpyAsync(L, b.L, (c->nr + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
    }
}

int run_diagnostics_checked(ffpic_ctx *c, uint32_t what, ffpic_diag *out, double *L,
                            const DiagBufs &b) {
    return guarded(c, [&] { run_diagnostics(c, what, out, L, b); });
}

}  // namespace ffpic

extern "C" {

int ffpic_create(const ffpic_desc *d, void *stream, ffpic_ctx **out) {
    if (!out) return FFPIC_EINVAL;
    *out = nullptr;
    std::string why = validate(d);
    if (!why.empty()) return FFPIC_EINVAL;
    ffpic_ctx *c = new (std::nothrow) ffpic_ctx();
    if (!c) return FFPIC_ENOMEM;
    int rc = guarded(c, [&] {
        c->stream = (hipStream_t)stream;
        HCHK(hipGetDevice(&c->device));
        setup_geometry(c, d);
        if (c->d.sort_interval == 0) {
            int si, rows, ppt;
            tuned_settings(d, &si, &rows, &ppt);
            c->d.sort_interval = si;
            c->fused_rows = rows;
            c->push_ppt = ppt;
        }
        {   // first row where the absorber's factor (in working precision) is below 1
            auto below1 = [&](double v) { return c->fp64 ? v != 1.0 : (float)v != 1.0f; };
            c->absorb_row0 = c->nr + 1;
            for (int i = 0; i <= c->nr; i++)
                if (below1(c->tab[T_LAMN][i]) || (i < c->nr && below1(c->tab[T_LAMH][i]))) {
                    c->absorb_row0 = i;
                    break;
                }
        }
        for (int t = 0; t < T_NTAB; t++) {
            const auto &h = c->tab[t];
            c->dtab64[t] = (double *)dmalloc(h.size() * sizeof(double));
            HCHK(hipMemcpy(c->dtab64[t], h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
            if (c->fp64) {
                c->dtab[t] = c->dtab64[t];
            } else {
                std::vector<float> f(h.begin(), h.end());
                c->dtab[t] = dmalloc(f.size() * sizeof(float));
                HCHK(hipMemcpy(c->dtab[t], f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
            }
        }
        size_t fb = c->nn * c->rsz;
        // the three components of a field are one allocation, cstride
        // elements apart (a kernel takes one base per field)
        c->cstride = (c->nn + 63) & ~size_t(63);
        alloc3(c, c->E, false);
        alloc3(c, c->B, false);
        alloc3(c, c->B0, false);
        alloc3(c, c->J, true);
        alloc3(c, c->Jalt, true);
        alloc3(c, c->stAlt, true);
        alloc3(c, c->stAlt + 3, true);
        c->psi = (double *)dmalloc(c->nn * sizeof(double));
        c->f = dmalloc(fb);
        c->kill = (uint8_t *)dmalloc((size_t)c->nr * c->nth);
        int64_t maxcap = 0;
        for (int s = 0; s < d->nspec; s++) {
            Species &S = c->sp[s];
            S.cap = d->capacity[s];
            S.qm = d->qm[s];
            S.weight = d->weight[s];
            S.narr = c->fp64 ? 5 : 6;
            size_t eb = c->fp64 ? 8 : 4;
            for (int a = 0; a < S.narr; a++) {
                S.cur[a] = dmalloc((size_t)S.cap * eb);
                S.alt[a] = dmalloc((size_t)S.cap * eb);
            }
            maxcap = std::max(maxcap, S.cap);
        }
        c->sort_cap = maxcap;
        for (int k = 0; k < 2; k++) {
            c->keys[k] = (uint32_t *)dmalloc((size_t)maxcap * 4);
            c->vals[k] = (uint32_t *)dmalloc((size_t)maxcap * 4);
        }
        sort_alloc(c, maxcap, dmalloc);
        {
            const size_t nk1 = (size_t)c->nr * c->nth + 1;
            c->sort_aux = (uint32_t *)dmalloc((size_t)std::max<int64_t>(maxcap, 1) * 4);
            c->sort_kcnt = (int32_t *)dmalloc(nk1 * 4);
            HCHK(hipMemset(c->sort_kcnt, 0, nk1 * 4));
            // room for the state of a quarter of the slots changing cell
            // between two sorts; the movers past it are read from their slots
            c->sort_cbuf_n = std::max<int64_t>(maxcap / 4, 1);
            c->sort_cbuf = dmalloc((size_t)c->sort_cbuf_n * (c->fp64 ? 5 * 8 : 6 * 4));

            for (int s = 0; s < d->nspec; s++)
                for (int k = 0; k < 2; k++) c->soff[s][k] = (int32_t *)dmalloc(nk1 * 4);
        }
        // scans: the movers per key of the sort, the surface sources' counts
        int64_t scan_n = std::max<int64_t>((int64_t)c->nr * c->nth + 1, c->nth + 1);
        if (d->gamma_th > 0.0) {
            const int64_t per = (maxcap + pair_block_slots() - 1) / pair_block_slots();
            c->pair_blocks = 2 * per;
            c->pair_cnt = (int32_t *)dmalloc((size_t)(c->pair_blocks + 1) * sizeof(int32_t));
            c->pair_off = (int32_t *)dmalloc((size_t)(c->pair_blocks + 1) * sizeof(int32_t));
            scan_n = std::max<int64_t>(scan_n, c->pair_blocks + 1);
        }
        c->scan_part_n = scan_part_len(scan_n);
        c->scan_part = (int32_t *)dmalloc((size_t)c->scan_part_n * sizeof(int32_t));
        c->nslots = (int32_t *)dmalloc(FFPIC_MAX_SPECIES * sizeof(int32_t));
        c->nalive = (int32_t *)dmalloc(FFPIC_MAX_SPECIES * sizeof(int32_t));
        c->nsorted = (int32_t *)dmalloc(FFPIC_MAX_SPECIES * sizeof(int32_t));
        c->removed = (unsigned long long *)dmalloc(FFPIC_MAX_SPECIES * 4 * sizeof(unsigned long long));
        c->err = (uint32_t *)dmalloc(sizeof(uint32_t));
        c->red_len = 4096;
        c->red = (double *)dmalloc(c->red_len * sizeof(double));
        HCHK(hipMemset(c->nslots, 0, FFPIC_MAX_SPECIES * sizeof(int32_t)));
        HCHK(hipMemset(c->nalive, 0, FFPIC_MAX_SPECIES * sizeof(int32_t)));
        HCHK(hipMemset(c->nsorted, 0, FFPIC_MAX_SPECIES * sizeof(int32_t)));
        HCHK(hipMemset(c->removed, 0, FFPIC_MAX_SPECIES * 4 * sizeof(unsigned long long)));
        HCHK(hipMemset(c->err, 0, sizeof(uint32_t)));
        for (auto &e : c->ev) HCHK(hipEventCreate(&e));
        std::vector<double> F[6];
        init_fields_host(c, F);
        surface_tables(c, F[3].data());   // row 0 of B_r: the stellar surface
        for (int k = 0; k < 3; k++) {
            upload_field(c, c->E[k], F[k]);
            upload_field(c, c->B[k], F[3 + k]);
            upload_field(c, c->B0[k], F[3 + k]);
        }
        if (!c->fp64) {
            alloc3(c, c->dE, true);
            alloc3(c, c->dB, true);
            alloc3(c, c->E0, false);
            alloc3(c, c->rE0, false);
            alloc3(c, c->rB0, false);
            for (int k = 0; k < 3; k++) {
                c->hE0[k] = F[k];
                c->hB0[k] = F[3 + k];
            }
            c->rho0 = dmalloc(fb);
            {
                std::vector<float> rowc, colc;
                fused32_tables(c, rowc, colc);
                c->fz_rowc = dmalloc(rowc.size() * sizeof(float));
                c->fz_colc = dmalloc(colc.size() * sizeof(float));
                HCHK(hipMemcpy(c->fz_rowc, rowc.data(), rowc.size() * sizeof(float), hipMemcpyHostToDevice));
                HCHK(hipMemcpy(c->fz_colc, colc.data(), colc.size() * sizeof(float), hipMemcpyHostToDevice));
            }
            for (int k = 0; k < 2; k++) {
                c->E0d[k] = (double *)dmalloc(c->nn * sizeof(double));
                c->B0d[k] = (double *)dmalloc(c->nn * sizeof(double));
            }
            upload_background(c);
        }
        psi_mask(c);
        HCHK(hipStreamSynchronize(c->stream));
    });
    if (rc != FFPIC_OK) {
        free_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return FFPIC_OK;
}

int ffpic_host_table(const ffpic_desc *d, int table, double *out, int64_t *n) {
    if (!validate(d).empty() || table < 0 || table >= T_NTAB || !n) return FFPIC_EINVAL;
    return guarded(nullptr, [&] {
        ffpic_ctx c;
        setup_geometry(&c, d);
        const auto &t = c.tab[table];
        if (out) std::copy(t.begin(), t.end(), out);
        *n = (int64_t)t.size();
    });
}

int ffpic_host_initial_field(const ffpic_desc *d, int comp, double *out) {
    if (!validate(d).empty() || comp < FFPIC_ER || comp > FFPIC_BPH || !out) return FFPIC_EINVAL;
    return guarded(nullptr, [&] {
        ffpic_ctx c;
        setup_geometry(&c, d);
        std::vector<double> F[6];
        init_fields_host(&c, F);
        std::copy(F[comp].begin(), F[comp].end(), out);
    });
}

void ffpic_destroy(ffpic_ctx *c) {
    if (!c || c->batch_owned) return;   // views are released with their batch
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

const char *ffpic_last_error(const ffpic_ctx *c) {
    if (!c) return "no context";
    return c->last_error.c_str();
}

int ffpic_info(const ffpic_ctx *c, double out[4]) {
    if (!c || !out) return FFPIC_EINVAL;
    out[0] = c->dt; out[1] = c->dlog; out[2] = c->dth; out[3] = c->omega;
    return FFPIC_OK;
}

int ffpic_load_fields(ffpic_ctx *c, int comp, const double *src, int on_dev) {
    return guarded(c, [&] {
        check_ctx(c);
        if (comp < FFPIC_ER || comp > FFPIC_BPH || !src) throw Fail{FFPIC_EINVAL, "bad component or NULL source"};
        void *dst = comp < 3 ? c->E[comp] : c->B[comp - 3];
        const double *dsrc = src;
        double *tmp = nullptr;
        if (!on_dev) {
            tmp = (double *)dmalloc(c->nn * sizeof(double));
            HCHK(hipMemcpyAsync(tmp, src, c->nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
            dsrc = tmp;
        }
        from_f64(c, dsrc, dst, c->nn);
        if (comp >= FFPIC_BR) from_f64(c, dsrc, c->B0[comp - 3], c->nn);
        if (comp == FFPIC_BR) {
            psi_mask(c);
            if (c->d.inject_kappa > 0.0) {
                std::vector<double> row(c->nth);
                HCHK(hipMemcpyAsync(row.data(), dsrc, (size_t)c->nth * sizeof(double),
                                    hipMemcpyDeviceToHost, c->stream));
                HCHK(hipStreamSynchronize(c->stream));
                surface_tables(c, row.data());
            }
        }
        if (!c->fp64) {
            // the loaded component becomes the background of that component
            std::vector<double> h(c->nn);
            HCHK(hipMemcpyAsync(h.data(), dsrc, c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HCHK(hipStreamSynchronize(c->stream));
            size_t fb = c->nn * sizeof(float);
            if (comp < 3) {
                c->hE0[comp] = h;
                HCHK(hipMemset(c->dE[comp], 0, fb));
            } else {
                c->hB0[comp - 3] = h;
                HCHK(hipMemset(c->dB[comp - 3], 0, fb));
            }
            upload_background(c);
        }
        HCHK(hipStreamSynchronize(c->stream));
        if (tmp) HCHK(hipFree(tmp));
    });
}

int ffpic_load_particles(ffpic_ctx *c, int s, int64_t n, const double *r, const double *th,
                         const double *ur, const double *uth, const double *uph, int on_dev) {
    return guarded(c, [&] {
        check_ctx(c);
        if (s < 0 || s >= c->d.nspec) throw Fail{FFPIC_EINVAL, "species out of range"};
        if (n < 0) throw Fail{FFPIC_EINVAL, "negative count"};
        if (n == 0) return;
        if (!r || !th || !ur || !uth || !uph) throw Fail{FFPIC_EINVAL, "NULL particle array"};
        Species &S = c->sp[s];
        if (S.nub + n > S.cap) throw Fail{FFPIC_ECAPACITY, "species capacity exceeded"};
        const double *src[5] = {r, th, ur, uth, uph};
        double *stage = nullptr;
        if (!on_dev) {
            stage = (double *)dmalloc((size_t)n * 5 * sizeof(double));
            for (int a = 0; a < 5; a++)
                HCHK(hipMemcpyAsync(stage + (size_t)a * n, src[a], (size_t)n * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream));
            for (int a = 0; a < 5; a++) src[a] = stage + (size_t)a * n;
        }
        convert_loaded(c, s, S.nub, n, src[0], src[1], src[2], src[3], src[4]);
        S.nub += n;
        c->sort_valid[s] = false;   // appended particles: full sort
        int32_t ns = (int32_t)S.nub;
        HCHK(hipMemcpyAsync(c->nslots + s, &ns, sizeof(ns), hipMemcpyHostToDevice, c->stream));
        sort_species(c, s);
        int32_t alive = 0;
        HCHK(hipMemcpyAsync(&alive, c->nslots + s, sizeof(alive), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        S.nub = alive;
        if (stage) HCHK(hipFree(stage));
    });
}

int ffpic_step(ffpic_ctx *c, int32_t nsteps) {
    return guarded(c, [&] {
        check_ctx(c);
        if (nsteps < 0) throw Fail{FFPIC_EINVAL, "negative step count"};
        if (c->timing) {
            for (auto &m : c->phase_ms) m = 0.f;
            while ((int)c->evpool.size() < 5 * nsteps) {
                hipEvent_t e;
                HCHK(hipEventCreate(&e));
                c->evpool.push_back(e);
            }
        }
        const int si = c->d.sort_interval;
        for (int k = 0; k < nsteps;) {
            // whole sort cycles as graphs, the other steps one by one
            if (c->step % si == 0 && nsteps - k >= si && cycle_graphable(c)) {
                run_cycle_graph(c, si);
                k += si;
                continue;
            }
            one_step(c, step_phases(c), true, c->timing ? k : -1);
            k++;
        }
        if (c->timing && nsteps > 0) {
            // events only: the stream is not drained between steps
            HCHK(hipEventSynchronize(c->evpool[5 * nsteps - 1]));
            for (int s = 0; s < nsteps; s++)
                for (int k = 0; k < 4; k++) {
                    float ms = 0;
                    HCHK(hipEventElapsedTime(&ms, c->evpool[5 * s + k], c->evpool[5 * s + k + 1]));
                    c->phase_ms[k] += ms;
                }
        }
    });
}

int ffpic_run_phases(ffpic_ctx *c, uint32_t ph) {
    return guarded(c, [&] {
        check_ctx(c);
        one_step(c, ph, false, -1);
    });
}

int ffpic_sync(ffpic_ctx *c) {
    return guarded(c, [&] {
        check_ctx(c);
        HCHK(hipStreamSynchronize(c->stream));
        read_err(c);
    });
}

int ffpic_get_field(ffpic_ctx *c, int comp, double *dst, int on_dev) {
    return guarded(c, [&] {
        check_ctx(c);
        if (comp < 0 || comp >= FFPIC_NCOMP || !dst) throw Fail{FFPIC_EINVAL, "bad component or NULL destination"};
        double *d = dst;
        double *tmp = nullptr;
        if (!on_dev) { tmp = (double *)dmalloc(c->nn * sizeof(double)); d = tmp; }
        switch (comp) {
        case FFPIC_ER: case FFPIC_ETH: case FFPIC_EPH: to_f64(c, c->E[comp], d, c->nn); break;
        case FFPIC_BR: case FFPIC_BTH: case FFPIC_BPH: to_f64(c, c->B[comp - 3], d, c->nn); break;
        case FFPIC_JR: case FFPIC_JTH: case FFPIC_JPH: to_f64(c, c->J[comp - 6], d, c->nn); break;
        case FFPIC_PSI: HCHK(hipMemcpyAsync(d, c->psi, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream)); break;
        case FFPIC_F: to_f64(c, c->f, d, c->nn); break;
        case FFPIC_GAUSS: {
            double *qn = (double *)dmalloc(c->nn * sizeof(double));
            gauss(c, qn, d, nullptr);
            HCHK(hipStreamSynchronize(c->stream));
            HCHK(hipFree(qn));
            break;
        }
        case FFPIC_DIVB: divb(c, d, nullptr); break;
        }
        if (tmp) {
            HCHK(hipMemcpyAsync(dst, tmp, c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        }
        HCHK(hipStreamSynchronize(c->stream));
        if (tmp) HCHK(hipFree(tmp));
        read_err(c);
    });
}

int ffpic_num_particles(ffpic_ctx *c, int s, int64_t *n) {
    return guarded(c, [&] {
        check_ctx(c);
        if (s < 0 || s >= c->d.nspec || !n) throw Fail{FFPIC_EINVAL, "bad species or NULL"};
        int32_t ns = 0;
        HCHK(hipMemcpyAsync(&ns, c->nslots + s, sizeof(ns), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        *n = ns;
    });
}

int ffpic_get_particles_range(ffpic_ctx *c, int s, int64_t first, int64_t *count, double *r,
                              double *th, double *ur, double *uth, double *uph, int32_t *cell) {
    return guarded(c, [&] {
        check_ctx(c);
        if (s < 0 || s >= c->d.nspec) throw Fail{FFPIC_EINVAL, "bad species"};
        if (!count || first < 0 || *count < 0) throw Fail{FFPIC_EINVAL, "bad range"};
        int32_t ns = 0;
        HCHK(hipMemcpyAsync(&ns, c->nslots + s, sizeof(ns), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        int64_t n = std::max<int64_t>(0, std::min<int64_t>(*count, (int64_t)ns - first));
        *count = n;
        if (n == 0) return;
        double *buf = (double *)dmalloc((size_t)n * (5 * sizeof(double) + sizeof(int32_t)));
        double *o[5];
        for (int a = 0; a < 5; a++) o[a] = buf + (size_t)a * n;
        int32_t *oc = (int32_t *)(buf + (size_t)5 * n);
        export_particles(c, s, first, n, o[0], o[1], o[2], o[3], o[4], oc);
        double *h[5] = {r, th, ur, uth, uph};
        for (int a = 0; a < 5; a++)
            if (h[a]) HCHK(hipMemcpyAsync(h[a], o[a], (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (cell) HCHK(hipMemcpyAsync(cell, oc, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        HCHK(hipFree(buf));
    });
}

int ffpic_get_particles(ffpic_ctx *c, int s, double *r, double *th, double *ur, double *uth,
                        double *uph, int32_t *cell) {
    int64_t count = INT64_MAX;
    return ffpic_get_particles_range(c, s, 0, &count, r, th, ur, uth, uph, cell);
}

int ffpic_get_sort(ffpic_ctx *c, int s, int32_t *off, int32_t *perm, int64_t *nperm) {
    return guarded(c, [&] {
        check_ctx(c);
        if (s < 0 || s >= c->d.nspec || !off) throw Fail{FFPIC_EINVAL, "bad species or NULL"};
        if ((perm || nperm) && !c->perm_valid[s])
            throw Fail{FFPIC_EINVAL, "the last sort of this species was not recorded "
                                     "(ffpic_record_sort)"};
        size_t nk = (size_t)c->nr * c->nth + 1;
        int32_t *d = (int32_t *)dmalloc(nk * sizeof(int32_t));
        sort_offsets(c, s, d);
        HCHK(hipMemcpyAsync(off, d, nk * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        HCHK(hipFree(d));
        if (perm || nperm) {
            // the live count right after that sort is the last cell offset it
            // recorded
            const int t = c->sort_cur[s];
            int32_t n = 0;
            HCHK(hipMemcpy(&n, c->soff[s][t] + (nk - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
            if (perm)
                HCHK(hipMemcpy(perm, c->perm[s], (size_t)n * sizeof(int32_t),
                               hipMemcpyDeviceToHost));
            if (nperm) *nperm = n;
        }
    });
}

int ffpic_record_sort(ffpic_ctx *c, int on) {
    return guarded(c, [&] {
        check_ctx(c);
        if (on) {
            for (int s = 0; s < c->d.nspec; s++)
                if (!c->perm[s])
                    c->perm[s] = (int32_t *)dmalloc((size_t)std::max<int64_t>(c->sp[s].cap, 1) *
                                                    sizeof(int32_t));
        }
        c->record_perm = on != 0;
    });
}

int ffpic_spectra(ffpic_ctx *c, int s, const ffpic_spectra_req *q, double *dN, double *sed,
                  double *prad) {
    return guarded(c, [&] {
        check_ctx(c);
        if (s < 0 || s >= c->d.nspec) throw Fail{FFPIC_EINVAL, "species out of range"};
        if (!q || !dN || !sed || !prad) throw Fail{FFPIC_EINVAL, "NULL request or output"};
        if (q->ngamma < 1 || q->ngamma > FFPIC_SPEC_MAX || q->nnu < 1 || q->nnu > FFPIC_SPEC_MAX)
            throw Fail{FFPIC_EINVAL, "ngamma and nnu must lie in [1, FFPIC_SPEC_MAX]"};
        if (!(q->rmin < q->rmax) || !(q->thmin < q->thmax))
            throw Fail{FFPIC_EINVAL, "empty region"};
        if (!(q->gmin > 0) || !(q->gmax > q->gmin) || !std::isfinite(q->gmax))
            throw Fail{FFPIC_EINVAL, "need 0 < gmin < gmax"};
        if (!(q->numin > 0) || !std::isfinite(q->numax) ||
            !(q->nnu == 1 ? q->numax >= q->numin : q->numax > q->numin))
            throw Fail{FFPIC_EINVAL, "need 0 < numin < numax"};
        const size_t len = (size_t)q->ngamma + q->nnu + 1;
        if (len > c->red_len) throw Fail{FFPIC_EINVAL, "request too large"};
        spectra(c, s, q, c->red);
        std::vector<double> h(len);
        HCHK(hipMemcpyAsync(h.data(), c->red, len * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        read_err(c);
        std::copy(h.begin(), h.begin() + q->ngamma, dN);
        std::copy(h.begin() + q->ngamma, h.begin() + q->ngamma + q->nnu, sed);
        *prad = h[len - 1];
    });
}

int ffpic_diagnostics(ffpic_ctx *c, uint32_t what, ffpic_diag *out, double *L) {
    return guarded(c, [&] {
        check_ctx(c);
        if (!out) throw Fail{FFPIC_EINVAL, "NULL output"};
        struct Owned {   // per-call device scratch, released on every path
            std::vector<void *> p;
            ~Owned() { for (void *q : p) (void)hipFree(q); }
            double *take(size_t n) { p.push_back(dmalloc(n * sizeof(double))); return (double *)p.back(); }
        } own;
        DiagBufs b;
        b.part = c->red;
        b.out = own.take(16);
        if (what & FFPIC_DIAG_RESIDUALS) b.qn = own.take(c->nn);
        if ((what & FFPIC_DIAG_POYNTING) && L) b.L = own.take(c->nr + 1);
        run_diagnostics(c, what, out, L, b);
        HCHK(hipStreamSynchronize(c->stream));
    });
}

// ---------------------------------------------------------------------------
// checkpoints: header, then raw device images of the state

namespace {
struct SaveHeader {
    char magic[8];
    uint32_t version, precision;
    int32_t nr, nth, nspec, pad;
    int64_t step;
    int64_t nslots[FFPIC_MAX_SPECIES];
    unsigned long long removed[FFPIC_MAX_SPECIES * 4];
    uint32_t err, pad2;
};

size_t save_size(ffpic_ctx *c, const int32_t *ns) {
    size_t fb = c->nn * c->rsz;
    size_t bytes = sizeof(SaveHeader) + 9 * fb + c->nn * sizeof(double) + fb;
    if (!c->fp64) bytes += 6 * fb + 6 * c->nn * sizeof(double);   // dE, dB, FP64 background
    for (int s = 0; s < c->d.nspec; s++)
        bytes += (size_t)ns[s] * (c->fp64 ? 5 * 8 : 6 * 4);
    return bytes;
}
}  // namespace

int ffpic_save(ffpic_ctx *c, void *buf, size_t *len) {
    return guarded(c, [&] {
        check_ctx(c);
        if (!len) throw Fail{FFPIC_EINVAL, "NULL length"};
        HCHK(hipStreamSynchronize(c->stream));
        int32_t ns[FFPIC_MAX_SPECIES] = {};
        HCHK(hipMemcpy(ns, c->nslots, sizeof(ns), hipMemcpyDeviceToHost));
        size_t need = save_size(c, ns);
        if (!buf) { *len = need; return; }
        if (*len < need) throw Fail{FFPIC_EINVAL, "checkpoint buffer too small"};
        SaveHeader h{};
        std::memcpy(h.magic, "FFPICSV1", 8);
        h.version = 1;
        h.precision = (uint32_t)c->d.precision;
        h.nr = c->nr; h.nth = c->nth; h.nspec = c->d.nspec;
        h.step = c->step;
        for (int s = 0; s < FFPIC_MAX_SPECIES; s++) h.nslots[s] = ns[s];
        HCHK(hipMemcpy(h.removed, c->removed, sizeof(h.removed), hipMemcpyDeviceToHost));
        HCHK(hipMemcpy(&h.err, c->err, sizeof(uint32_t), hipMemcpyDeviceToHost));
        char *p = (char *)buf;
        std::memcpy(p, &h, sizeof(h));
        p += sizeof(h);
        size_t fb = c->nn * c->rsz;
        void *arrs[9] = {c->E[0], c->E[1], c->E[2], c->B[0], c->B[1], c->B[2], c->B0[0], c->B0[1], c->B0[2]};
        for (void *a : arrs) { HCHK(hipMemcpy(p, a, fb, hipMemcpyDeviceToHost)); p += fb; }
        HCHK(hipMemcpy(p, c->psi, c->nn * sizeof(double), hipMemcpyDeviceToHost)); p += c->nn * sizeof(double);
        HCHK(hipMemcpy(p, c->f, fb, hipMemcpyDeviceToHost)); p += fb;
        if (!c->fp64) {
            for (int k = 0; k < 3; k++) {
                HCHK(hipMemcpy(p, c->dE[k], fb, hipMemcpyDeviceToHost)); p += fb;
                HCHK(hipMemcpy(p, c->dB[k], fb, hipMemcpyDeviceToHost)); p += fb;
            }
            for (int k = 0; k < 3; k++) {
                std::memcpy(p, c->hE0[k].data(), c->nn * sizeof(double)); p += c->nn * sizeof(double);
                std::memcpy(p, c->hB0[k].data(), c->nn * sizeof(double)); p += c->nn * sizeof(double);
            }
        }
        size_t eb = c->fp64 ? 8 : 4;
        for (int s = 0; s < c->d.nspec; s++)
            for (int a = 0; a < c->sp[s].narr; a++) {
                HCHK(hipMemcpy(p, c->sp[s].cur[a], (size_t)ns[s] * eb, hipMemcpyDeviceToHost));
                p += (size_t)ns[s] * eb;
            }
        *len = need;
    });
}

int ffpic_restore(ffpic_ctx *c, const void *buf, size_t len) {
    return guarded(c, [&] {
        check_ctx(c);
        if (!buf || len < sizeof(SaveHeader)) throw Fail{FFPIC_EINVAL, "checkpoint too short"};
        SaveHeader h;
        std::memcpy(&h, buf, sizeof(h));
        if (std::memcmp(h.magic, "FFPICSV1", 8) != 0 || h.version != 1)
            throw Fail{FFPIC_EINVAL, "not a checkpoint of this library"};
        if (h.precision != (uint32_t)c->d.precision || h.nr != c->nr || h.nth != c->nth ||
            h.nspec != c->d.nspec)
            throw Fail{FFPIC_EINVAL, "checkpoint does not match this context"};
        int32_t ns[FFPIC_MAX_SPECIES] = {};
        for (int s = 0; s < FFPIC_MAX_SPECIES; s++) ns[s] = (int32_t)h.nslots[s];
        for (int s = 0; s < c->d.nspec; s++)
            if (ns[s] > c->sp[s].cap) throw Fail{FFPIC_ECAPACITY, "checkpoint exceeds capacity"};
        if (len < save_size(c, ns)) throw Fail{FFPIC_EINVAL, "checkpoint truncated"};
        HCHK(hipStreamSynchronize(c->stream));
        const char *p = (const char *)buf + sizeof(h);
        size_t fb = c->nn * c->rsz;
        void *arrs[9] = {c->E[0], c->E[1], c->E[2], c->B[0], c->B[1], c->B[2], c->B0[0], c->B0[1], c->B0[2]};
        for (void *a : arrs) { HCHK(hipMemcpy(a, p, fb, hipMemcpyHostToDevice)); p += fb; }
        HCHK(hipMemcpy(c->psi, p, c->nn * sizeof(double), hipMemcpyHostToDevice)); p += c->nn * sizeof(double);
        HCHK(hipMemcpy(c->f, p, fb, hipMemcpyHostToDevice)); p += fb;
        if (!c->fp64) {
            for (int k = 0; k < 3; k++) {
                HCHK(hipMemcpy(c->dE[k], p, fb, hipMemcpyHostToDevice)); p += fb;
                HCHK(hipMemcpy(c->dB[k], p, fb, hipMemcpyHostToDevice)); p += fb;
            }
            for (int k = 0; k < 3; k++) {
                c->hE0[k].assign((const double *)p, (const double *)p + c->nn); p += c->nn * sizeof(double);
                c->hB0[k].assign((const double *)p, (const double *)p + c->nn); p += c->nn * sizeof(double);
            }
            upload_background(c);
        }
        size_t eb = c->fp64 ? 8 : 4;
        for (int s = 0; s < c->d.nspec; s++) {
            for (int a = 0; a < c->sp[s].narr; a++) {
                HCHK(hipMemcpy(c->sp[s].cur[a], p, (size_t)ns[s] * eb, hipMemcpyHostToDevice));
                p += (size_t)ns[s] * eb;
            }
            c->sp[s].nub = ns[s];
        }
        HCHK(hipMemcpy(c->nslots, ns, sizeof(ns), hipMemcpyHostToDevice));
        HCHK(hipMemcpy(c->removed, h.removed, sizeof(h.removed), hipMemcpyHostToDevice));
        for (int s = 0; s < FFPIC_MAX_SPECIES; s++) c->sort_valid[s] = false;
        HCHK(hipMemcpy(c->err, &h.err, sizeof(uint32_t), hipMemcpyHostToDevice));
        for (int k = 0; k < 3; k++) HCHK(hipMemset(c->J[k], 0, fb));
        // the kill flags follow from Psi
        psi_mask(c);
        HCHK(hipStreamSynchronize(c->stream));
        c->step = h.step;
    });
}

int ffpic_set_field_rows(ffpic_ctx *c, int32_t rows) {
    return guarded(c, [&] {
        check_ctx(c);
        if (rows < 0) throw Fail{FFPIC_EINVAL, "negative row count"};
        c->fused_rows = rows;
    });
}

int ffpic_set_push_chunk(ffpic_ctx *c, int32_t ppt) {
    return guarded(c, [&] {
        check_ctx(c);
        if (ppt != 8 && ppt != 16 && ppt != 32)
            throw Fail{FFPIC_EINVAL, "particles per thread must be 8, 16 or 32"};
        c->push_ppt = ppt;
    });
}

int ffpic_set_graph(ffpic_ctx *c, int on) {
    return guarded(c, [&] {
        check_ctx(c);
        c->use_graph = on != 0;
        if (!c->use_graph) destroy_graphs(c);
    });
}

int ffpic_graph_stats(ffpic_ctx *c, int64_t *builds, int64_t *launches) {
    if (!c) return FFPIC_EINVAL;
    if (builds) *builds = c->graph_builds;
    if (launches) *launches = c->graph_launches;
    return FFPIC_OK;
}

int ffpic_set_timing(ffpic_ctx *c, int enable) {
    if (!c) return FFPIC_EINVAL;
    c->timing = enable ? 1 : 0;
    return FFPIC_OK;
}

int ffpic_phase_times(ffpic_ctx *c, float out[4]) {
    if (!c || !out) return FFPIC_EINVAL;
    for (int k = 0; k < 4; k++) out[k] = c->phase_ms[k];
    return FFPIC_OK;
}

}  // extern "C"

namespace ffpic {

void steps_one_by_one(ffpic_ctx *c, int n) {
    for (int k = 0; k < n; k++) one_step(c, step_phases(c), true, -1);
}

bool graphable_cycle(const ffpic_ctx *c) { return cycle_graphable(c); }

bool step_sorts(const ffpic_ctx *c) { return (step_phases(c) & FFPIC_PHASE_SORT) != 0; }

CycleState get_cycle_state(const ffpic_ctx *c) { return cycle_state(c); }

void put_cycle_state(ffpic_ctx *c, const CycleState &st) { set_cycle_state(c, st); }

double rr_factor(const ffpic_ctx *c) {
#pragma clang fp contract(off)
    return rr_factor_at(c->d, (double)c->step * c->dt);
}

}  // namespace ffpic
