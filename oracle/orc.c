/*
 * FP64 CPU oracle for distance-preconditioned Wilson-clover inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes (de Divitiis, Petronzio, Tantalo, "Distance
 * preconditioning for lattice Dirac operators"):
 *
 *  - the lattice Dirac system (D[U] + M) S = eta          (eq. linsysunprec)
 *  - D[U] is the O(a)-improved Wilson operator (section on heavy quarks):
 *        D = 1/2 sum_mu { gamma_mu (nabla_mu + nabla*_mu) - nabla*_mu nabla_mu }
 *            + c_sw (i/4) sum_{mu,nu} sigma_mu_nu Fhat_mu_nu
 *    with the covariant derivatives exactly as the paper writes them
 *        nabla_mu  S(y) = U_mu(y) S(y+mu) - S(y)
 *        nabla*_mu S(y) = S(y) - U_mu(y-mu)^+ S(y-mu)
 *    sigma_mu_nu = (i/2)[gamma_mu, gamma_nu], Fhat = (Q_mu_nu - Q_nu_mu)/8,
 *    Q the sum of the four plaquette leaves at y in the (mu,nu) plane.
 *    The paper names the operator but prints no formula for it; this is the
 *    standard form it refers to.  Chiral gamma basis, gamma5 = diag(1,1,-1,-1).
 *  - the field redefinition (eq. redeft) and the preconditioned operator
 *    (eq. linsysprec), in the convention S' = alpha S, eta' = alpha eta
 *    (alpha here is the reciprocal of the function the paper factorises),
 *    computed two ways:
 *      literal:   D' psi' = alpha (D + M) (alpha^-1 psi')
 *      modified:  D + M with the time derivatives replaced by the modified
 *                 ones (the paper's modified nabla_0, nabla*_0) and the
 *                 boundary rule of eq. redeftbc for the field S'.
 *  - the light-quark generalisation (eqs. redefa, betaa, redefcovs): the
 *    redefinition by beta(y) = prod_mu alpha_mu(y_mu), one profile per
 *    direction, literally beta (D+M) beta^-1, and through the modified
 *    covariant derivatives in all four directions with the boundary rule of
 *    eq. redeftbc applied in each direction;
 *  - the global stopping rule |(D'+M) S' - eta'| < r (eq. stopping), read as
 *    the L2 norm relative to |eta'|;
 *  - BiCGStab (van der Vorst 1992) and CG on the normal equations;
 *  - restoration S = S'/alpha and the correlator
 *        C_PP(y0) = - sum_{vec y} tr[S^+(y) S(y)]
 *    (section on heavy quarks), indexed by t = (y0 - x0_src) mod T.
 *
 * Time boundary of the fermion: antiperiodic, periodic, or Dirichlet (bc_t =
 * 0: the field vanishes beyond the first and last timeslice, so the hops
 * across the boundary drop; the fermion boundary of the Schroedinger
 * functional with zero boundary fields, for which the paper used the
 * exponential profile).
 *
 * Layouts (complex128 interleaved, x0 slowest, x3 fastest):
 *   U[site][mu][a][b], psi[site][spin][colour], C[site][12][12]
 *   with row/column index 3*spin + colour.  dims = {T, L1, L2, L3}.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOCONV -3
#define ORC_EBREAK -4

typedef struct {
    int L[4];
    long V;
    int bc_t; /* +1 periodic, -1 antiperiodic, 0 Dirichlet in time for the fermion */
} lattice;

/* ---------------------------------------------------------------- geometry */

static long site_of(const lattice *g, const int x[4])
{
    return (((long)x[0] * g->L[1] + x[1]) * g->L[2] + x[2]) * g->L[3] + x[3];
}

static void coords_of(const lattice *g, long s, int x[4])
{
    for (int mu = 3; mu >= 0; --mu) {
        x[mu] = (int)(s % g->L[mu]);
        s /= g->L[mu];
    }
}

/* site reached from s by one step (+1 or -1) along mu; *crossed is set when
 * the step wraps around the lattice in that direction */
static long step_of(const lattice *g, long s, int mu, int dir, int *crossed)
{
    int x[4];
    coords_of(g, s, x);
    x[mu] += dir;
    *crossed = 0;
    if (x[mu] >= g->L[mu]) { x[mu] -= g->L[mu]; *crossed = 1; }
    if (x[mu] < 0) { x[mu] += g->L[mu]; *crossed = 1; }
    return site_of(g, x);
}

static int setup(lattice *g, const int dims[4], int bc_t)
{
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 1) return ORC_EINVAL;
        g->L[mu] = dims[mu];
    }
    if (bc_t != 1 && bc_t != -1 && bc_t != 0) return ORC_EINVAL;
    g->V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    g->bc_t = bc_t;
    return ORC_OK;
}

/* ------------------------------------------------------- Dirac matrices */

static cplx gam[4][4][4]; /* gam[mu][row][col], chiral basis */
static cplx sig[4][4][4][4]; /* sig[mu][nu] = (i/2)[gamma_mu, gamma_nu] */
static int gam_ready = 0;

static void init_gammas(void)
{
    if (gam_ready) return;
    memset(gam, 0, sizeof gam);
    /* gamma_0 = [[0,-1],[-1,0]] in 2x2 blocks */
    gam[0][0][2] = -1; gam[0][1][3] = -1; gam[0][2][0] = -1; gam[0][3][1] = -1;
    /* gamma_k = [[0,-i sigma_k],[i sigma_k,0]] with the Pauli matrices */
    const cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                gam[k + 1][a][b + 2] = -I * pauli[k][a][b];
                gam[k + 1][a + 2][b] = I * pauli[k][a][b];
            }
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k)
                        c += gam[mu][a][k] * gam[nu][k][b] - gam[nu][a][k] * gam[mu][k][b];
                    sig[mu][nu][a][b] = 0.5 * I * c;
                }
    gam_ready = 1;
}

/* ------------------------------------------------------- small helpers */

static const cplx *link(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

static void mat_mul(const cplx *A, const cplx *B, cplx *C) /* C = A B, 3x3 */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx c = 0;
            for (int k = 0; k < 3; ++k) c += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = c;
        }
}

static void mat_dag(const cplx *A, cplx *B)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i * 3 + j] = conj(A[j * 3 + i]);
}

/* out = A psi (colour matrix on each spin component), or A^+ psi */
static void colour_mul(const cplx *A, int dagger, const cplx *psi, cplx *out)
{
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx c = 0;
            for (int b = 0; b < 3; ++b)
                c += (dagger ? conj(A[b * 3 + a]) : A[a * 3 + b]) * psi[s * 3 + b];
            out[s * 3 + a] = c;
        }
}

/* ---------------------------------------------------------------- clover */

/* Q_mu_nu(x): sum of the four plaquette leaves in the (mu,nu) plane that
 * start and end at x, all with the same orientation. */
static void clover_leaves(const lattice *g, const cplx *U, long x, int mu, int nu, cplx *Q)
{
    int c;
    long xpm = step_of(g, x, mu, +1, &c), xmm = step_of(g, x, mu, -1, &c);
    long xpn = step_of(g, x, nu, +1, &c), xmn = step_of(g, x, nu, -1, &c);
    long xmm_pn = step_of(g, xmm, nu, +1, &c), xmm_mn = step_of(g, xmm, nu, -1, &c);
    long xpm_mn = step_of(g, xpm, nu, -1, &c);
    cplx A[9], B[9], Cm[9], D[9], t1[9], t2[9], leaf[9];

    memset(Q, 0, 9 * sizeof(cplx));
    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
    memcpy(A, link(U, x, mu), sizeof A);
    memcpy(B, link(U, xpm, nu), sizeof B);
    mat_dag(link(U, xpn, mu), Cm);
    mat_dag(link(U, x, nu), D);
    mat_mul(A, B, t1); mat_mul(t1, Cm, t2); mat_mul(t2, D, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
    /* U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
    memcpy(A, link(U, x, nu), sizeof A);
    mat_dag(link(U, xmm_pn, mu), B);
    mat_dag(link(U, xmm, nu), Cm);
    memcpy(D, link(U, xmm, mu), sizeof D);
    mat_mul(A, B, t1); mat_mul(t1, Cm, t2); mat_mul(t2, D, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
    /* U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
    mat_dag(link(U, xmm, mu), A);
    mat_dag(link(U, xmm_mn, nu), B);
    memcpy(Cm, link(U, xmm_mn, mu), sizeof Cm);
    memcpy(D, link(U, xmn, nu), sizeof D);
    mat_mul(A, B, t1); mat_mul(t1, Cm, t2); mat_mul(t2, D, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
    /* U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+ */
    mat_dag(link(U, xmn, nu), A);
    memcpy(B, link(U, xmn, mu), sizeof B);
    memcpy(Cm, link(U, xpm_mn, nu), sizeof Cm);
    mat_dag(link(U, x, mu), D);
    mat_mul(A, B, t1); mat_mul(t1, Cm, t2); mat_mul(t2, D, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
}

/* C(x) = c_sw (i/4) sum_{mu,nu} sigma_mu_nu (x) Fhat_mu_nu(x), as a dense
 * 12x12 matrix per site (row 3*spin+colour). */
int orc_clover(const int dims[4], const double *U_, double csw, double *C_)
{
    lattice g;
    if (setup(&g, dims, -1) != ORC_OK) return ORC_EINVAL;
    init_gammas();
    const cplx *U = (const cplx *)U_;
    cplx *C = (cplx *)C_;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g.V; ++x) {
        cplx *Cx = C + x * 144;
        memset(Cx, 0, 144 * sizeof(cplx));
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                if (mu == nu) continue;
                cplx Qmn[9], Qnm[9], F[9];
                clover_leaves(&g, U, x, mu, nu, Qmn);
                clover_leaves(&g, U, x, nu, mu, Qnm);
                for (int i = 0; i < 9; ++i) F[i] = (Qmn[i] - Qnm[i]) / 8.0;
                for (int s = 0; s < 4; ++s)
                    for (int t = 0; t < 4; ++t) {
                        cplx w = csw * 0.25 * I * sig[mu][nu][s][t];
                        if (w == 0) continue;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                Cx[(s * 3 + a) * 12 + t * 3 + b] += w * F[a * 3 + b];
                    }
            }
    }
    return ORC_OK;
}

/* ------------------------------------------------- the Dirac operator */

/*
 * Factors of the covariant derivatives, per direction.  fwd[mu][x_mu]
 * multiplies U_mu(y) S(y+mu) in nabla_mu at y_mu = x_mu, bwd[mu][x_mu]
 * multiplies U_mu(y-mu)^+ S(y-mu) in nabla*_mu; both include the fermion
 * boundary sign where the step crosses the boundary (time only: space is
 * periodic).  A NULL direction carries the boundary sign only.
 */
typedef struct {
    const double *fwd[4], *bwd[4];
} hop_factors;

/* (D + M) psi with the derivative definitions above; C may be NULL (c_sw=0).
 * hf == NULL: plain derivatives with the boundary sign only. */
static void dirac_nabla(const lattice *g, const cplx *U, const cplx *C, double M,
                        const hop_factors *hf, const cplx *in, cplx *out)
{
    const long V = g->V;
    cplx *dpsi = malloc(sizeof(cplx) * 12 * V); /* nabla_mu psi, one mu at a time */
    double *fwdm[4], *bwdm[4];
    for (int mu = 0; mu < 4; ++mu) {
        const int L = g->L[mu];
        const double sign = mu == 0 ? g->bc_t : 1.0;
        fwdm[mu] = malloc(sizeof(double) * L);
        bwdm[mu] = malloc(sizeof(double) * L);
        for (int t = 0; t < L; ++t) {
            if (hf && hf->fwd[mu]) { fwdm[mu][t] = hf->fwd[mu][t]; bwdm[mu][t] = hf->bwd[mu][t]; }
            else {
                fwdm[mu][t] = (t == L - 1) ? sign : 1.0;
                bwdm[mu][t] = (t == 0) ? sign : 1.0;
            }
        }
    }

#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx *o = out + 12 * x;
        const cplx *p = in + 12 * x;
        for (int i = 0; i < 12; ++i) o[i] = M * p[i];
        if (C) {
            const cplx *Cx = C + 144 * x;
            for (int i = 0; i < 12; ++i) {
                cplx c = 0;
                for (int j = 0; j < 12; ++j) c += Cx[i * 12 + j] * p[j];
                o[i] += c;
            }
        }
    }

    for (int mu = 0; mu < 4; ++mu) {
        /* dpsi = nabla_mu psi */
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            int cr, xc[4];
            long xp = step_of(g, x, mu, +1, &cr);
            coords_of(g, x, xc);
            const double f = fwdm[mu][xc[mu]];
            cplx tmp[12];
            colour_mul(link(U, x, mu), 0, in + 12 * xp, tmp);
            for (int i = 0; i < 12; ++i) dpsi[12 * x + i] = f * tmp[i] - in[12 * x + i];
        }
        /* out += 1/2 [ gamma_mu (nabla + nabla*) psi - nabla*(nabla psi) ] */
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            int cr, xc[4];
            long xm = step_of(g, x, mu, -1, &cr);
            coords_of(g, x, xc);
            const double b = bwdm[mu][xc[mu]];
            cplx back_psi[12], back_d[12], ds[12], lap[12];
            colour_mul(link(U, xm, mu), 1, in + 12 * xm, back_psi);
            colour_mul(link(U, xm, mu), 1, dpsi + 12 * xm, back_d);
            /* Dirichlet time boundary: psi vanishes on the slice before x0 = 0, but
             * its forward derivative there, U psi(x), does not; U^+ of it is psi(x) */
            const int virt = mu == 0 && g->bc_t == 0 && xc[0] == 0;
            for (int i = 0; i < 12; ++i) {
                cplx nab_star = in[12 * x + i] - b * back_psi[i];
                ds[i] = dpsi[12 * x + i] + nab_star;           /* (nabla + nabla*) psi */
                lap[i] = dpsi[12 * x + i] - (virt ? in[12 * x + i] : b * back_d[i]); /* nabla*(nabla psi) */
            }
            cplx *o = out + 12 * x;
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx gs = 0;
                    for (int t = 0; t < 4; ++t) gs += gam[mu][s][t] * ds[t * 3 + a];
                    o[s * 3 + a] += 0.5 * (gs - lap[s * 3 + a]);
                }
        }
    }
    free(dpsi);
    for (int mu = 0; mu < 4; ++mu) { free(fwdm[mu]); free(bwdm[mu]); }
}

/* gamma5 = diag(1,1,-1,-1) in this basis */
static void apply_g5(long V, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x)
        for (int i = 0; i < 12; ++i) out[12 * x + i] = (i < 6 ? 1.0 : -1.0) * in[12 * x + i];
}

/* the redefinition factor at site x: beta(x) = prod_mu prof[mu][x_mu]
 * (eq. betaa's product form; a NULL direction contributes 1, and with only
 * prof[0] set this is the time-only alpha of eq. redeft) */
static double beta_at(const lattice *g, const double *const prof[4], long x)
{
    int xc[4];
    coords_of(g, x, xc);
    double b = 1.0;
    for (int mu = 0; mu < 4; ++mu)
        if (prof[mu]) b *= prof[mu][xc[mu]];
    return b;
}

static void scale_by_beta(const lattice *g, const double *const prof[4], int inverse, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g->V; ++x) {
        const double b = beta_at(g, prof, x);
        const double f = inverse ? 1.0 / b : b;
        for (int i = 0; i < 12; ++i) out[12 * x + i] = f * in[12 * x + i];
    }
}

typedef struct {
    lattice g;
    const cplx *U, *C;
    double M;
    const double *prof[4]; /* all NULL: no preconditioning */
    cplx *tmp;
} op_ctx;

/* literal preconditioned operator: D' psi = beta (D+M) beta^-1 psi */
static void op_prec(op_ctx *o, const cplx *in, cplx *out)
{
    scale_by_beta(&o->g, o->prof, 1, in, o->tmp);
    dirac_nabla(&o->g, o->U, o->C, o->M, NULL, o->tmp, out);
    scale_by_beta(&o->g, o->prof, 0, out, out);
}

/* its adjoint: D'^+ = beta^-1 (D+M)^+ beta, with (D+M)^+ = gamma5 (D+M) gamma5 */
static void op_prec_dag(op_ctx *o, const cplx *in, cplx *out)
{
    scale_by_beta(&o->g, o->prof, 0, in, o->tmp);
    apply_g5(o->g.V, o->tmp, o->tmp);
    dirac_nabla(&o->g, o->U, o->C, o->M, NULL, o->tmp, out);
    apply_g5(o->g.V, out, out);
    scale_by_beta(&o->g, o->prof, 1, out, out);
}

static int check_profile(int L, const double *a)
{
    if (!a) return ORC_OK;
    for (int t = 0; t < L; ++t)
        if (!(a[t] > 0) || !isfinite(a[t])) return ORC_EINVAL;
    return ORC_OK;
}

static int check_alpha(int T, const double *alpha) { return check_profile(T, alpha); }

/* prof4: NULL, or T + L1 + L2 + L3 values (the four profiles one after the other) */
static int split_profiles(const lattice *g, const double *prof4, const double *prof[4])
{
    long off = 0;
    for (int mu = 0; mu < 4; ++mu) {
        prof[mu] = prof4 ? prof4 + off : NULL;
        if (check_profile(g->L[mu], prof[mu])) return ORC_EINVAL;
        off += g->L[mu];
    }
    return ORC_OK;
}

/* out = D' in (dagger = 0) or D'^+ in (dagger = 1); alpha NULL means alpha = 1 */
int orc_apply(const int dims[4], int bc_t, const double *U, const double *C, double M,
              const double *alpha, int dagger, const double *in, double *out)
{
    op_ctx o;
    if (setup(&o.g, dims, bc_t) != ORC_OK || check_alpha(dims[0], alpha)) return ORC_EINVAL;
    init_gammas();
    o.U = (const cplx *)U; o.C = (const cplx *)C; o.M = M;
    o.prof[0] = alpha; o.prof[1] = o.prof[2] = o.prof[3] = NULL;
    o.tmp = malloc(sizeof(cplx) * 12 * o.g.V);
    if (!o.tmp) return ORC_ENOMEM;
    if (dagger) op_prec_dag(&o, (const cplx *)in, (cplx *)out);
    else op_prec(&o, (const cplx *)in, (cplx *)out);
    free(o.tmp);
    return ORC_OK;
}

/* out = D' in or D'^+ in for beta(y) = prod_mu alpha_mu(y_mu) (eq. redefa);
 * prof4 = T + L1 + L2 + L3 profile values (NULL: beta = 1) */
int orc_apply_beta(const int dims[4], int bc_t, const double *U, const double *C, double M,
                   const double *prof4, int dagger, const double *in, double *out)
{
    op_ctx o;
    if (setup(&o.g, dims, bc_t) != ORC_OK || split_profiles(&o.g, prof4, o.prof)) return ORC_EINVAL;
    init_gammas();
    o.U = (const cplx *)U; o.C = (const cplx *)C; o.M = M;
    o.tmp = malloc(sizeof(cplx) * 12 * o.g.V);
    if (!o.tmp) return ORC_ENOMEM;
    if (dagger) op_prec_dag(&o, (const cplx *)in, (cplx *)out);
    else op_prec(&o, (const cplx *)in, (cplx *)out);
    free(o.tmp);
    return ORC_OK;
}

/*
 * D' + M through the modified time derivatives: at y0 the forward derivative
 * carries alpha(y0)/alpha(y0+1) in front of U_0(y) S'(y+0) and the backward
 * one alpha(y0)/alpha(y0-1) in front of U_0(y-0)^+ S'(y-0) (this is the
 * paper's rule with its function replaced by the reciprocal).  Where y0+1 = T
 * or y0-1 = -1 the field S' beyond the boundary is taken from eq. redeftbc,
 * which needs alpha outside [0, T): alpha_T = alpha(T) and alpha_m1 =
 * alpha(-1) are that extension.  In this convention the rule reads
 *   S'(y + T 0) = bc_t * alpha(y0 + T) / alpha(y0) * S'(y).
 */
int orc_apply_modified(const int dims[4], int bc_t, const double *U, const double *C, double M,
                       const double *alpha, double alpha_T, double alpha_m1,
                       const double *in, double *out)
{
    lattice g;
    if (setup(&g, dims, bc_t) != ORC_OK || check_alpha(dims[0], alpha) || !alpha) return ORC_EINVAL;
    if (!(alpha_T > 0) || !(alpha_m1 > 0)) return ORC_EINVAL;
    init_gammas();
    const int T = dims[0];
    double *fwd = malloc(sizeof(double) * T), *bwd = malloc(sizeof(double) * T);
    for (int t = 0; t < T; ++t) {
        if (t + 1 < T) fwd[t] = alpha[t] / alpha[t + 1];
        else {
            /* ratio to the extended alpha times the boundary rule S'(T) = bc alpha(T)/alpha(0) S'(0) */
            fwd[t] = alpha[t] / alpha_T * (bc_t * alpha_T / alpha[0]);
        }
        if (t > 0) bwd[t] = alpha[t] / alpha[t - 1];
        else {
            /* S'(-1) = bc alpha(-1)/alpha(T-1) S'(T-1) */
            bwd[t] = alpha[t] / alpha_m1 * (bc_t * alpha_m1 / alpha[T - 1]);
        }
    }
    hop_factors hf = {{fwd, NULL, NULL, NULL}, {bwd, NULL, NULL, NULL}};
    dirac_nabla(&g, (const cplx *)U, (const cplx *)C, M, &hf, (const cplx *)in, (cplx *)out);
    free(fwd); free(bwd);
    return ORC_OK;
}

/*
 * D' + M for beta(y) = prod_mu alpha_mu(y_mu) through the modified covariant
 * derivatives of eq. redefcovs in every direction (reciprocal convention as
 * above): nabla_mu carries alpha_mu(y_mu)/alpha_mu(y_mu+1), nabla*_mu carries
 * alpha_mu(y_mu)/alpha_mu(y_mu-1), and beyond the boundary in direction mu the
 * field is continued as eq. redeftbc continues it in time,
 *   S'(y + L_mu mu) = s_mu * alpha_mu(y_mu + L_mu) / alpha_mu(y_mu) * S'(y),
 * with s_mu the fermion's boundary sign (bc_t in time, +1 in space) and the
 * extension values ext[2 mu] = alpha_mu(L_mu), ext[2 mu + 1] = alpha_mu(-1).
 */
int orc_apply_modified4(const int dims[4], int bc_t, const double *U, const double *C, double M,
                        const double *prof4, const double *ext, const double *in, double *out)
{
    lattice g;
    const double *prof[4];
    if (setup(&g, dims, bc_t) != ORC_OK || !prof4 || !ext || split_profiles(&g, prof4, prof)) return ORC_EINVAL;
    for (int k = 0; k < 8; ++k)
        if (!(ext[k] > 0)) return ORC_EINVAL;
    init_gammas();
    double *fwd[4], *bwd[4];
    for (int mu = 0; mu < 4; ++mu) {
        const int L = dims[mu];
        const double sign = mu == 0 ? bc_t : 1.0;
        const double *a = prof[mu];
        fwd[mu] = malloc(sizeof(double) * L);
        bwd[mu] = malloc(sizeof(double) * L);
        for (int t = 0; t < L; ++t) {
            if (t + 1 < L) fwd[mu][t] = a[t] / a[t + 1];
            else fwd[mu][t] = a[t] / ext[2 * mu] * (sign * ext[2 * mu] / a[0]);
            if (t > 0) bwd[mu][t] = a[t] / a[t - 1];
            else bwd[mu][t] = a[t] / ext[2 * mu + 1] * (sign * ext[2 * mu + 1] / a[L - 1]);
        }
    }
    hop_factors hf = {{fwd[0], fwd[1], fwd[2], fwd[3]}, {bwd[0], bwd[1], bwd[2], bwd[3]}};
    dirac_nabla(&g, (const cplx *)U, (const cplx *)C, M, &hf, (const cplx *)in, (cplx *)out);
    for (int mu = 0; mu < 4; ++mu) { free(fwd[mu]); free(bwd[mu]); }
    return ORC_OK;
}

/* ------------------------------------------------------------- solvers */

static cplx dot(long n, const cplx *a, const cplx *b) /* sum conj(a) b */
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; ++i) {
        cplx c = conj(a[i]) * b[i];
        re += creal(c); im += cimag(c);
    }
    return re + I * im;
}

static double norm2(long n, const cplx *a) { return creal(dot(n, a, a)); }

/* BiCGStab (van der Vorst 1992) for D' x = b, x starts at 0; stops when
 * |b - D' x| <= r |b| on the recursively updated residual, then the caller
 * recomputes the true residual. */
static int bicgstab(op_ctx *o, const cplx *b, cplx *x, double rtol, int maxit, int *iters)
{
    const long n = 12 * o->g.V;
    cplx *r = calloc(n, sizeof(cplx)), *rh = calloc(n, sizeof(cplx)), *p = calloc(n, sizeof(cplx));
    cplx *v = calloc(n, sizeof(cplx)), *s = calloc(n, sizeof(cplx)), *t = calloc(n, sizeof(cplx));
    if (!r || !rh || !p || !v || !s || !t) return ORC_ENOMEM;
    memset(x, 0, n * sizeof(cplx));
    memcpy(r, b, n * sizeof(cplx));
    memcpy(rh, b, n * sizeof(cplx));
    const double bn = sqrt(norm2(n, b));
    cplx rho = 1, alpha = 1, omega = 1;
    int k = 0, restarts = 0, status = ORC_ENOCONV;
    if (bn == 0) { status = ORC_OK; goto done; }
    for (k = 0; k < maxit; ++k) {
        if (sqrt(norm2(n, r)) <= rtol * bn) { status = ORC_OK; break; }
        cplx rho_new = dot(n, rh, r);
        if (cabs(rho_new) <= 1e-14 * sqrt(norm2(n, rh) * norm2(n, r))) {
            /* (near) breakdown: restart from the current iterate with the
             * current residual as the new shadow residual */
            if (restarts++ > 20) { status = ORC_EBREAK; break; }
            memcpy(rh, r, n * sizeof(cplx));
            memset(p, 0, n * sizeof(cplx));
            memset(v, 0, n * sizeof(cplx));
            rho = alpha = omega = 1;
            rho_new = dot(n, rh, r);
        }
        cplx beta = (rho_new / rho) * (alpha / omega);
        rho = rho_new;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        op_prec(o, p, v);
        alpha = rho / dot(n, rh, v);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        op_prec(o, s, t);
        double tt = norm2(n, t);
        if (tt == 0) { /* s is already the residual of the converged iterate */
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] = s[i]; }
            continue;
        }
        omega = dot(n, t, s) / tt;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
    }
    if (k == maxit && sqrt(norm2(n, r)) <= rtol * bn) status = ORC_OK;
done:
    *iters = k;
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return status;
}

/* CG on the normal equations D'^+ D' x = D'^+ b (Hestenes-Stiefel), tracking
 * the residual of the original system r = b - D' x. */
static int cgnr(op_ctx *o, const cplx *b, cplx *x, double rtol, int maxit, int *iters)
{
    const long n = 12 * o->g.V;
    cplx *r = calloc(n, sizeof(cplx)), *z = calloc(n, sizeof(cplx));
    cplx *p = calloc(n, sizeof(cplx)), *w = calloc(n, sizeof(cplx));
    if (!r || !z || !p || !w) return ORC_ENOMEM;
    memset(x, 0, n * sizeof(cplx));
    memcpy(r, b, n * sizeof(cplx));
    const double bn = sqrt(norm2(n, b));
    int k = 0, status = ORC_ENOCONV;
    op_prec_dag(o, r, z);
    memcpy(p, z, n * sizeof(cplx));
    double zz = norm2(n, z);
    for (k = 0; k < maxit; ++k) {
        if (sqrt(norm2(n, r)) <= rtol * bn) { status = ORC_OK; break; }
        op_prec(o, p, w);
        double a = zz / norm2(n, w);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) { x[i] += a * p[i]; r[i] -= a * w[i]; }
        op_prec_dag(o, r, z);
        double zz_new = norm2(n, z);
        double beta = zz_new / zz;
        zz = zz_new;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (k == maxit && sqrt(norm2(n, r)) <= rtol * bn) status = ORC_OK;
    *iters = k;
    free(r); free(z); free(p); free(w);
    return status;
}

/*
 * Solve (D+M) S = eta through the preconditioned system:
 *   eta' = alpha eta, solve D' S' = eta' to |eta' - D'S'| <= r |eta'|,
 *   S = S' / alpha.
 * solver: 0 BiCGStab, 1 CGNR.  Sp (nullable) receives S'.  info[0] = iterations,
 * info[1] = true relative residual of the preconditioned system, info[2] = true
 * relative residual of the unpreconditioned system.
 */
static int solve_prof(op_ctx *po, int solver, const double *eta, double rtol, int maxit,
                      double *S, double *Sp, double *info);

int orc_solve(const int dims[4], int bc_t, const double *U, const double *C, double M,
              const double *alpha, int solver, const double *eta, double rtol, int maxit,
              double *S, double *Sp, double *info)
{
    op_ctx o;
    if (setup(&o.g, dims, bc_t) != ORC_OK || check_alpha(dims[0], alpha)) return ORC_EINVAL;
    o.U = (const cplx *)U; o.C = (const cplx *)C; o.M = M;
    o.prof[0] = alpha; o.prof[1] = o.prof[2] = o.prof[3] = NULL;
    return solve_prof(&o, solver, eta, rtol, maxit, S, Sp, info);
}

/* the same with beta(y) = prod_mu alpha_mu(y_mu): eta' = beta eta, S = S'/beta
 * (eqs. redefa, betaa; the restoration precedes any contraction) */
int orc_solve_beta(const int dims[4], int bc_t, const double *U, const double *C, double M,
                   const double *prof4, int solver, const double *eta, double rtol, int maxit,
                   double *S, double *Sp, double *info)
{
    op_ctx o;
    if (setup(&o.g, dims, bc_t) != ORC_OK || split_profiles(&o.g, prof4, o.prof)) return ORC_EINVAL;
    o.U = (const cplx *)U; o.C = (const cplx *)C; o.M = M;
    return solve_prof(&o, solver, eta, rtol, maxit, S, Sp, info);
}

static int solve_prof(op_ctx *po, int solver, const double *eta, double rtol, int maxit,
                      double *S, double *Sp, double *info)
{
    op_ctx o = *po;
    if (solver != 0 && solver != 1) return ORC_EINVAL;
    init_gammas();
    const long n = 12 * o.g.V;
    o.tmp = malloc(sizeof(cplx) * n);
    cplx *ep = malloc(sizeof(cplx) * n), *xp = malloc(sizeof(cplx) * n), *res = malloc(sizeof(cplx) * n);
    if (!o.tmp || !ep || !xp || !res) return ORC_ENOMEM;
    scale_by_beta(&o.g, o.prof, 0, (const cplx *)eta, ep);
    int iters = 0;
    int st = solver == 0 ? bicgstab(&o, ep, xp, rtol, maxit, &iters) : cgnr(&o, ep, xp, rtol, maxit, &iters);
    /* true residuals */
    op_prec(&o, xp, res);
    double en = sqrt(norm2(n, ep)), rn;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) res[i] = ep[i] - res[i];
    rn = sqrt(norm2(n, res));
    if (Sp) memcpy(Sp, xp, n * sizeof(cplx));
    scale_by_beta(&o.g, o.prof, 1, xp, (cplx *)S);
    op_ctx plain = o;
    plain.prof[0] = plain.prof[1] = plain.prof[2] = plain.prof[3] = NULL;
    op_prec(&plain, (const cplx *)S, res);
    const cplx *e = (const cplx *)eta;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) res[i] = e[i] - res[i];
    if (info) {
        info[0] = iters;
        info[1] = en > 0 ? rn / en : 0;
        double e0 = sqrt(norm2(n, e));
        info[2] = e0 > 0 ? sqrt(norm2(n, res)) / e0 : 0;
    }
    free(o.tmp); free(ep); free(xp); free(res);
    return st;
}

/*
 * The Schwarz alternating procedure with GCR, the solver of the paper's
 * light-quark iteration counts (Table 1; Luescher's domain-decomposition
 * method, which the paper cites), on the beta-preconditioned operator D'.
 *
 * The lattice is cut into blocks of extents bs[mu] (an even number of blocks
 * per direction) coloured by the parity of the block coordinates, so blocks
 * that touch have different colours.  One SAP application M r:
 *     psi = 0
 *     ncy times, for colour 0 then colour 1:
 *         rho = (r - D' psi) restricted to the blocks of that colour
 *         nmr minimal-residual steps on every block of that colour, with the
 *         block operator D'_B = P_B D' P_B (Dirichlet block boundaries):
 *             a = D'_B rho,  w_B = <a, rho>_B / <a, a>_B,
 *             psi += w_B rho,  rho -= w_B a
 * (while rho vanishes off the colour, P_c D' rho on the colour's sites is
 * exactly the direct sum of the block operators, since a block's neighbours
 * have the other colour).  GCR solves D' x = eta with this preconditioner on
 * the right: z_k = M r, w_k = D' z_k orthogonalised against the earlier w_j
 * (coefficients c_jk, norms b_k), r -= <w_k, r> w_k; after nkv steps or at
 * convergence x += sum_k a_k z_k with the triangular system of the c_jk and
 * b_k, and r is recomputed as eta - D' x.  Iterations count M applications.
 */
typedef struct {
    int bs[4];
    int nb[4];
    long nblocks;
} blocking;

static int setup_blocking(const lattice *g, const int bs[4], blocking *b)
{
    b->nblocks = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (bs[mu] < 1 || g->L[mu] % bs[mu]) return ORC_EINVAL;
        b->bs[mu] = bs[mu];
        b->nb[mu] = g->L[mu] / bs[mu];
        if (b->nb[mu] % 2) return ORC_EINVAL; /* touching blocks must differ in colour */
        b->nblocks *= b->nb[mu];
    }
    return ORC_OK;
}

static long block_of(const lattice *g, const blocking *b, long x, int *colour)
{
    int xc[4];
    coords_of(g, x, xc);
    long k = 0;
    int sum = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const int c = xc[mu] / b->bs[mu];
        k = k * b->nb[mu] + c;
        sum += c;
    }
    *colour = sum & 1;
    return k;
}

/* nmr minimal-residual steps on the blocks of one colour: psi += sum w_B rho */
static void sap_blocks(op_ctx *o, const blocking *b, const long *blk, const int *col, int colour, int nmr,
                       cplx *rho, cplx *a, cplx *psi, cplx *num, double *den)
{
    const long V = o->g.V;
    for (int k = 0; k < nmr; ++k) {
        op_prec(o, rho, a);
        for (long q = 0; q < b->nblocks; ++q) { num[q] = 0; den[q] = 0; }
        for (long x = 0; x < V; ++x) {
            if (col[x] != colour) continue;
            cplx nm = 0;
            double dn = 0;
            for (int i = 0; i < 12; ++i) {
                nm += conj(a[12 * x + i]) * rho[12 * x + i];
                dn += creal(conj(a[12 * x + i]) * a[12 * x + i]);
            }
            num[blk[x]] += nm;
            den[blk[x]] += dn;
        }
        for (long x = 0; x < V; ++x) {
            if (col[x] != colour) continue;
            const cplx w = den[blk[x]] > 0 ? num[blk[x]] / den[blk[x]] : 0;
            for (int i = 0; i < 12; ++i) {
                psi[12 * x + i] += w * rho[12 * x + i];
                rho[12 * x + i] -= w * a[12 * x + i];
            }
        }
    }
}

/* psi = M r */
static void sap_apply(op_ctx *o, const blocking *b, const long *blk, const int *col, int ncy, int nmr,
                      const cplx *r, cplx *psi, cplx *rho, cplx *a, cplx *num, double *den)
{
    const long n = 12 * o->g.V;
    memset(psi, 0, sizeof(cplx) * n);
    for (int cy = 0; cy < ncy; ++cy)
        for (int colour = 0; colour < 2; ++colour) {
            op_prec(o, psi, a);
            for (long x = 0; x < o->g.V; ++x)
                for (int i = 0; i < 12; ++i)
                    rho[12 * x + i] = col[x] == colour ? r[12 * x + i] - a[12 * x + i] : 0;
            sap_blocks(o, b, blk, col, colour, nmr, rho, a, psi, num, den);
        }
}

static int sap_gcr(op_ctx *o, const blocking *b, int ncy, int nmr, int nkv, const cplx *eta, cplx *x,
                   double rtol, int maxit, int *iters)
{
    const long V = o->g.V, n = 12 * V;
    long *blk = malloc(sizeof(long) * V);
    int *col = malloc(sizeof(int) * V);
    cplx *r = malloc(sizeof(cplx) * n), *rho = malloc(sizeof(cplx) * n), *a = malloc(sizeof(cplx) * n);
    cplx *z = malloc(sizeof(cplx) * n * nkv), *w = malloc(sizeof(cplx) * n * nkv);
    cplx *num = malloc(sizeof(cplx) * b->nblocks), *cc = malloc(sizeof(cplx) * nkv * nkv);
    cplx *gam = malloc(sizeof(cplx) * nkv), *al = malloc(sizeof(cplx) * nkv);
    double *den = malloc(sizeof(double) * b->nblocks), *bn = malloc(sizeof(double) * nkv);
    if (!blk || !col || !r || !rho || !a || !z || !w || !num || !cc || !gam || !al || !den || !bn) return ORC_ENOMEM;
    for (long s = 0; s < V; ++s) blk[s] = block_of(&o->g, b, s, &col[s]);
    memset(x, 0, sizeof(cplx) * n);
    memcpy(r, eta, sizeof(cplx) * n);
    const double target = rtol * sqrt(norm2(n, eta));
    int it = 0, status = ORC_ENOCONV;
    double rn = sqrt(norm2(n, r));
    if (rn <= target) status = ORC_OK;
    while (status != ORC_OK && it < maxit) {
        int k = 0;
        for (; k < nkv && it < maxit; ++k) {
            cplx *zk = z + n * k, *wk = w + n * k;
            sap_apply(o, b, blk, col, ncy, nmr, r, zk, rho, a, num, den);
            op_prec(o, zk, wk);
            ++it;
            for (int j = 0; j < k; ++j) {
                const cplx *wj = w + n * j;
                const cplx c = dot(n, wj, wk);
                cc[j * nkv + k] = c;
                for (long i = 0; i < n; ++i) wk[i] -= c * wj[i];
            }
            bn[k] = sqrt(norm2(n, wk));
            if (!(bn[k] > 0)) { status = ORC_EBREAK; break; }
            for (long i = 0; i < n; ++i) wk[i] /= bn[k];
            gam[k] = dot(n, wk, r);
            for (long i = 0; i < n; ++i) r[i] -= gam[k] * wk[i];
            rn = sqrt(norm2(n, r));
            if (rn <= target) { ++k; break; }
        }
        if (status == ORC_EBREAK) break;
        /* the coefficients of the z_k: upper-triangular solve */
        for (int j = k - 1; j >= 0; --j) {
            cplx s = gam[j];
            for (int l = j + 1; l < k; ++l) s -= cc[j * nkv + l] * al[l];
            al[j] = s / bn[j];
        }
        for (int j = 0; j < k; ++j)
            for (long i = 0; i < n; ++i) x[i] += al[j] * z[n * j + i];
        op_prec(o, x, a);
        for (long i = 0; i < n; ++i) r[i] = eta[i] - a[i];
        rn = sqrt(norm2(n, r));
        if (rn <= target) status = ORC_OK;
    }
    *iters = it;
    free(blk); free(col); free(r); free(rho); free(a); free(z); free(w); free(num); free(cc);
    free(gam); free(al); free(den); free(bn);
    return status;
}

/* Solve (D+M) S = eta with SAP+GCR on the beta-preconditioned system
 * (prof4: NULL or the T + L1 + L2 + L3 profile values); par = {bs0..bs3,
 * ncy, nmr, nkv}.  info as for orc_solve. */
int orc_solve_sap(const int dims[4], int bc_t, const double *U, const double *C, double M, const double *prof4,
                  const int par[7], const double *eta, double rtol, int maxit, double *S, double *Sp, double *info)
{
    op_ctx o;
    blocking b;
    if (setup(&o.g, dims, bc_t) != ORC_OK || split_profiles(&o.g, prof4, o.prof)) return ORC_EINVAL;
    if (setup_blocking(&o.g, par, &b) != ORC_OK || par[4] < 1 || par[5] < 1 || par[6] < 1) return ORC_EINVAL;
    init_gammas();
    o.U = (const cplx *)U; o.C = (const cplx *)C; o.M = M;
    const long n = 12 * o.g.V;
    o.tmp = malloc(sizeof(cplx) * n);
    cplx *ep = malloc(sizeof(cplx) * n), *xp = malloc(sizeof(cplx) * n), *res = malloc(sizeof(cplx) * n);
    if (!o.tmp || !ep || !xp || !res) return ORC_ENOMEM;
    scale_by_beta(&o.g, o.prof, 0, (const cplx *)eta, ep);
    int iters = 0;
    int st = sap_gcr(&o, &b, par[4], par[5], par[6], ep, xp, rtol, maxit, &iters);
    op_prec(&o, xp, res);
    for (long i = 0; i < n; ++i) res[i] = ep[i] - res[i];
    const double en = sqrt(norm2(n, ep)), rn = sqrt(norm2(n, res));
    if (Sp) memcpy(Sp, xp, n * sizeof(cplx));
    scale_by_beta(&o.g, o.prof, 1, xp, (cplx *)S);
    if (info) {
        info[0] = iters;
        info[1] = en > 0 ? rn / en : 0;
        info[2] = 0;
    }
    free(o.tmp); free(ep); free(xp); free(res);
    return st;
}

/* psi = M r (one SAP application), for checking the preconditioner */
int orc_sap_apply(const int dims[4], int bc_t, const double *U, const double *C, double M, const double *prof4,
                  const int par[7], const double *r, double *psi)
{
    op_ctx o;
    blocking b;
    if (setup(&o.g, dims, bc_t) != ORC_OK || split_profiles(&o.g, prof4, o.prof)) return ORC_EINVAL;
    if (setup_blocking(&o.g, par, &b) != ORC_OK || par[4] < 1 || par[5] < 1) return ORC_EINVAL;
    init_gammas();
    o.U = (const cplx *)U; o.C = (const cplx *)C; o.M = M;
    const long V = o.g.V, n = 12 * V;
    o.tmp = malloc(sizeof(cplx) * n);
    long *blk = malloc(sizeof(long) * V);
    int *col = malloc(sizeof(int) * V);
    cplx *rho = malloc(sizeof(cplx) * n), *a = malloc(sizeof(cplx) * n), *num = malloc(sizeof(cplx) * b.nblocks);
    double *den = malloc(sizeof(double) * b.nblocks);
    if (!o.tmp || !blk || !col || !rho || !a || !num || !den) return ORC_ENOMEM;
    for (long s = 0; s < V; ++s) blk[s] = block_of(&o.g, &b, s, &col[s]);
    sap_apply(&o, &b, blk, col, par[4], par[5], (const cplx *)r, (cplx *)psi, rho, a, num, den);
    free(o.tmp); free(blk); free(col); free(rho); free(a); free(num); free(den);
    return ORC_OK;
}

/* C_PP(t) = - sum_{vec y} sum over the given columns of sum_{spin,colour} |S|^2,
 * t = (y0 - x0_src) mod T.  S: [ncols][V][12]. */
int orc_cpp(const int dims[4], int ncols, const double *S_, int x0_src, double *cpp)
{
    lattice g;
    if (setup(&g, dims, -1) != ORC_OK || ncols < 0) return ORC_EINVAL;
    const cplx *S = (const cplx *)S_;
    const int T = dims[0];
    const long per_t = g.V / T;
    for (int y0 = 0; y0 < T; ++y0) {
        double acc = 0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
        for (long k = 0; k < (long)ncols * per_t; ++k) {
            long c = k / per_t, xs = k % per_t;
            const cplx *p = S + (c * g.V + (long)y0 * per_t + xs) * 12;
            for (int i = 0; i < 12; ++i) acc += creal(conj(p[i]) * p[i]);
        }
        cpp[((y0 - x0_src) % T + T) % T] = -acc;
    }
    return ORC_OK;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* export the Dirac matrices so tests can check the Clifford algebra */
void orc_gamma(int mu, double *out /* 4x4 complex */)
{
    init_gammas();
    memcpy(out, gam[mu], sizeof(cplx) * 16);
}
