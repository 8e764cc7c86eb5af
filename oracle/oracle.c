/*
 * FP64 CPU oracle for three- and four-phonon scattering rates.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition of the per-mode rate, as in the
 * paper's CPU-only algorithm (Appendix, Algorithm 1: loop over the partners of
 * one mode, test energy conservation, accumulate WP and WP*|Vp|^2, then scale by
 * 1/nptk and const/nptk), generalised to both three-phonon signs and the three
 * four-phonon types.  The paper prints only the absorption weight; the other
 * weights, the matrix element, the prefactors and the units follow the standard
 * Fermi-golden-rule forms that the paper builds on (Methodology section):
 *
 *   n(w)   = 1/expm1(hbar w / kB T)
 *   G(D)   = exp(-D^2/sigma^2)/(sigma sqrt(pi))                      (Alg. 1, WP)
 *   V      = sum_t sum_{alpha...} Phi_t^{alpha...}/sqrt(prod M)
 *              * eps_0(a_0)_{alpha_0} prod_{r>=1} eps_r(a_r)_{alpha_r}
 *              * exp(i sum_{r>=1} Q_r . R_{t,r})
 *            with Q_r = s_r q_r and eps_r = e (s_r = +1) or conj(e) (s_r = -1)
 *   Gamma3 = (pi hbar / 4N)    sum w |V|^2 occ G / (w w' w'')
 *   Gamma4 = (pi hbar^2 / 8N^2) sum w |V|^2 occ G / (w w' w'' w''')
 *   WP3 = (1/N) sum w occ G/(w w' w''),   WP4 = (1/N^2) sum w occ G/(w w' w'' w''')
 *
 *   type  signs(s1,s2[,s3])  Delta                 occ                                 w (ordered sum)
 *   3+    (+,-)              w+w1-w2               n1-n2                               1
 *   3-    (-,-)              w-w1-w2               1+n1+n2                             1/2
 *   4++   (+,+,-)            w+w1+w2-w3            n1 n2 (1+n3) - (1+n1)(1+n2) n3      1/2
 *   4+-   (+,-,-)            w+w1-w2-w3            n1 (1+n2)(1+n3) - (1+n1) n2 n3      1/2
 *   4--   (-,-,-)            w-w1-w2-w3            (1+n1)(1+n2)(1+n3) - n1 n2 n3       1/6
 *
 * Momentum: q + sum_r Q_r = 0 mod G fixes the last partner.  A candidate is kept
 * iff |Delta| <= nsigma*sigma (Alg. 1 filter) and every mode has w >= omega_floor.
 * The filter's Delta is evaluated left to right with the partners of equal sign
 * in ascending global mode index, so the decision does not depend on the order
 * in which the partners are listed.
 *
 * Two modes: "brute" loops over every ordered partner tuple and applies the
 * filter itself; "list" evaluates a given list of triangle-reduced records, whose
 * weights follow from index equality (1, 1/2, 1/6).  Per-mode sums are
 * Neumaier-compensated.
 *
 * The paper prints none of the absolute prefactors (pi hbar/4, pi hbar^2/8 and
 * the 1/2, 1/6 weights).  They are pinned by a second derivation: the
 * golden-rule transition rates of the supercell Hamiltonian (1/m!) sum Phi u..u,
 * linearised in the row mode's occupation, equal this file's per-record rate for
 * every process type (distinct partners); the 1/2, 1/6 weights of repeated
 * partners are the ordered-sum convention, pinned by brute ordered sums equal to
 * triangle-list sums.  The adaptive width (process_sigma) is this build's reading
 * of a formula the paper names but does not print: it is pinned against its own
 * definition (quadrature of the mismatch spread), not against the paper.
 *
 * Units: amu, Angstrom, ps; omega in rad/ps; Phi in eV/Angstrom^m; Gamma in 1/ps.
 * Build: plain C11, no fast-math, no FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* SI 2019 exact h, kB, e; CODATA 2018 atomic mass constant */
#define SI_H 6.62607015e-34
#define SI_KB 1.380649e-23
#define SI_AMU 1.66053906660e-27
#define SI_EV 1.602176634e-19

/* unit of energy amu*A^2/ps^2 in J, of action amu*A^2/ps in J*s */
#define U_ENERGY (SI_AMU * 1e-20 / 1e-24)
#define U_ACTION (SI_AMU * 1e-20 / 1e-12)

static double c_hbar(void) { return SI_H / (2.0 * M_PI) / U_ACTION; }
static double c_kb(void) { return SI_KB / U_ENERGY; }
static double c_ev(void) { return SI_EV / U_ENERGY; }
/* kappa unit amu*A/ps^3/K in W/(m K) */
static double c_kappa(void) { return SI_AMU * 1e-10 / 1e-36; }

typedef struct {
    int32_t mesh[3];
    int32_t n_atoms;
    const double* masses; /* [n_atoms] amu */
    const double* omega;  /* [nq*nb] rad/ps, g = iq*nb + j */
    const double* evec;   /* [nq*nb][nb] complex as (re, im) pairs */
    double omega_floor;
    int64_t n3;
    const int32_t* atoms3; /* [n3][3] */
    const int32_t* cells3; /* [n3][2][3] */
    const double* phi3;    /* [n3][27] */
    int64_t n4;
    const int32_t* atoms4; /* [n4][4] */
    const int32_t* cells4; /* [n4][3][3] */
    const double* phi4;    /* [n4][81] */
    /* broadening: adaptive = 0 uses the fixed sigma of each call; adaptive = 1
     * uses sigma_p = max(factor * sigma0_p, sigma), see process_sigma */
    int32_t adaptive;
    double factor;
    const double* vel;     /* [nq*nb][3] group velocities, A/ps */
    double recip[9];       /* reciprocal vectors b_1..b_3 as rows, rad/A */
} orc_sys;

typedef struct {
    double re, im;
} cplx;

static cplx cmul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

/* Neumaier compensated accumulator */
typedef struct {
    double s, c;
} ksum;

static void kadd(ksum* k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static double kval(const ksum* k) { return k->s + k->c; }

/* OpenMP threads the rate sums use */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* thread count of the rate sums that follow (n > 0) */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_constants(double out[4]) {
    out[0] = c_hbar();
    out[1] = c_kb();
    out[2] = c_ev();
    out[3] = c_kappa();
}

double orc_bose(double omega, double T) { return 1.0 / expm1(c_hbar() * omega / (c_kb() * T)); }

double orc_gauss(double delta, double sigma) {
    return exp(-(delta * delta) / (sigma * sigma)) / (sigma * sqrt(M_PI));
}

static int64_t n_q(const orc_sys* s) { return (int64_t)s->mesh[0] * s->mesh[1] * s->mesh[2]; }

static int64_t wrap(int64_t x, int64_t n) { return ((x % n) + n) % n; }

/* mesh index of integer coordinates (any integers, reduced mod the mesh) */
static int64_t q_index(const orc_sys* s, const int64_t c[3]) {
    return (wrap(c[0], s->mesh[0]) * s->mesh[1] + wrap(c[1], s->mesh[1])) * s->mesh[2] +
           wrap(c[2], s->mesh[2]);
}

static void q_coords(const orc_sys* s, int64_t iq, int64_t c[3]) {
    c[2] = iq % s->mesh[2];
    c[1] = (iq / s->mesh[2]) % s->mesh[1];
    c[0] = iq / ((int64_t)s->mesh[1] * s->mesh[2]);
}

static int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* exp(i 2 pi sum_d k_d / N_d) for integer k_d, reduced exactly before the cosine */
static cplx root_of_unity(const orc_sys* s, const int64_t k[3]) {
    int64_t L = s->mesh[0];
    L = L / gcd64(L, s->mesh[1]) * s->mesh[1];
    L = L / gcd64(L, s->mesh[2]) * s->mesh[2];
    int64_t num = 0;
    for (int d = 0; d < 3; ++d) num += wrap(k[d], s->mesh[d]) * (L / s->mesh[d]);
    num = wrap(num, L);
    double ang = 2.0 * M_PI * (double)num / (double)L;
    cplx r = {cos(ang), sin(ang)};
    return r;
}

static cplx evec_at(const orc_sys* s, int64_t g, int comp, int sign) {
    int nb = 3 * s->n_atoms;
    const double* p = s->evec + 2 * (g * nb + comp);
    cplx r = {p[0], sign > 0 ? p[1] : -p[1]};
    return r;
}

/*
 * Matrix element of order m (3 or 4) for slots r = 0..m-1 at integer mesh
 * coordinates qc[r] (signed wavevector Q_r = sg[r]*qc[r]), branches br[r].
 * Slot 0 sits in the home cell of every term.
 */
static cplx vertex(const orc_sys* s, int m, const int64_t qc[][3], const int32_t* br, const int32_t* sg) {
    int nb = 3 * s->n_atoms;
    int64_t n_terms = m == 3 ? s->n3 : s->n4;
    const int32_t* atoms = m == 3 ? s->atoms3 : s->atoms4;
    const int32_t* cells = m == 3 ? s->cells3 : s->cells4;
    const double* phi = m == 3 ? s->phi3 : s->phi4;
    int ncomp = m == 3 ? 27 : 81;
    int64_t g[4];
    for (int r = 0; r < m; ++r) g[r] = q_index(s, qc[r]) * nb + br[r];
    double ev = c_ev();
    cplx V = {0.0, 0.0};
    for (int64_t t = 0; t < n_terms; ++t) {
        const int32_t* at = atoms + t * m;
        const int32_t* ce = cells + t * (m - 1) * 3;
        const double* ph = phi + t * ncomp;
        /* phase exp(i sum_{r>=1} Q_r . R_{t,r}) */
        int64_t k[3] = {0, 0, 0};
        for (int r = 1; r < m; ++r)
            for (int d = 0; d < 3; ++d) k[d] += (int64_t)sg[r] * qc[r][d] * ce[(r - 1) * 3 + d];
        cplx phase = root_of_unity(s, k);
        double msc = 1.0;
        for (int r = 0; r < m; ++r) msc *= s->masses[at[r]];
        double scale = ev / sqrt(msc);
        cplx acc = {0.0, 0.0};
        if (m == 3) {
            for (int a0 = 0; a0 < 3; ++a0) {
                cplx p0 = evec_at(s, g[0], 3 * at[0] + a0, sg[0]);
                for (int a1 = 0; a1 < 3; ++a1) {
                    cplx p1 = cmul(p0, evec_at(s, g[1], 3 * at[1] + a1, sg[1]));
                    for (int a2 = 0; a2 < 3; ++a2) {
                        cplx p2 = cmul(p1, evec_at(s, g[2], 3 * at[2] + a2, sg[2]));
                        double f = ph[(a0 * 3 + a1) * 3 + a2];
                        acc.re += f * p2.re;
                        acc.im += f * p2.im;
                    }
                }
            }
        } else {
            for (int a0 = 0; a0 < 3; ++a0) {
                cplx p0 = evec_at(s, g[0], 3 * at[0] + a0, sg[0]);
                for (int a1 = 0; a1 < 3; ++a1) {
                    cplx p1 = cmul(p0, evec_at(s, g[1], 3 * at[1] + a1, sg[1]));
                    for (int a2 = 0; a2 < 3; ++a2) {
                        cplx p2 = cmul(p1, evec_at(s, g[2], 3 * at[2] + a2, sg[2]));
                        for (int a3 = 0; a3 < 3; ++a3) {
                            cplx p3 = cmul(p2, evec_at(s, g[3], 3 * at[3] + a3, sg[3]));
                            double f = ph[((a0 * 3 + a1) * 3 + a2) * 3 + a3];
                            acc.re += f * p3.re;
                            acc.im += f * p3.im;
                        }
                    }
                }
            }
        }
        cplx term = cmul(phase, acc);
        V.re += scale * term.re;
        V.im += scale * term.im;
    }
    return V;
}

/* exported single matrix element; qc is [m][3] int32, br [m], sg [m] */
int orc_vertex(const orc_sys* s, int m, const int32_t* qc, const int32_t* br, const int32_t* sg, double* out) {
    if (m != 3 && m != 4) return -1;
    int64_t c[4][3];
    for (int r = 0; r < m; ++r)
        for (int d = 0; d < 3; ++d) c[r][d] = qc[r * 3 + d];
    cplx V = vertex(s, m, (const int64_t(*)[3])c, br, sg);
    out[0] = V.re;
    out[1] = V.im;
    return 0;
}

/* process types, shared numbering with the library interface */
enum { T3P = 0, T3M = 1, T4PP = 2, T4PM = 3, T4MM = 4 };

static int type_order(int ptype) { return ptype <= T3M ? 3 : 4; }

static void type_signs(int ptype, int32_t sg[4]) {
    sg[0] = 1;
    switch (ptype) {
        case T3P: sg[1] = 1; sg[2] = -1; break;
        case T3M: sg[1] = -1; sg[2] = -1; break;
        case T4PP: sg[1] = 1; sg[2] = 1; sg[3] = -1; break;
        case T4PM: sg[1] = 1; sg[2] = -1; sg[3] = -1; break;
        default: sg[1] = -1; sg[2] = -1; sg[3] = -1; break;
    }
}

/* occupation factor of a process type, difference form */
static double occupation(int ptype, const double* n) {
    switch (ptype) {
        case T3P: return n[1] - n[2];
        case T3M: return 1.0 + n[1] + n[2];
        case T4PP: return n[1] * n[2] * (1.0 + n[3]) - (1.0 + n[1]) * (1.0 + n[2]) * n[3];
        case T4PM: return n[1] * (1.0 + n[2]) * (1.0 + n[3]) - (1.0 + n[1]) * n[2] * n[3];
        default: return (1.0 + n[1]) * (1.0 + n[2]) * (1.0 + n[3]) - n[1] * n[2] * n[3];
    }
}

/* exported for the detailed-balance test; n[0] is the mode's own occupation */
double orc_occupation(int ptype, const double* n) { return occupation(ptype, n); }

/* ordered-sum weight of a type */
static double ordered_weight(int ptype) {
    if (ptype == T3P) return 1.0;
    if (ptype == T4MM) return 1.0 / 6.0;
    return 0.5;
}

/* weight of a triangle-reduced record, from equality of the interchangeable partners */
static double triangle_weight(int ptype, const int64_t* g) {
    switch (ptype) {
        case T3P: return 1.0;
        case T3M: return g[1] == g[2] ? 0.5 : 1.0;
        case T4PP: return g[1] == g[2] ? 0.5 : 1.0;
        case T4PM: return g[2] == g[3] ? 0.5 : 1.0;
        default:
            if (g[1] == g[2] && g[2] == g[3]) return 1.0 / 6.0;
            if (g[1] == g[2] || g[2] == g[3] || g[1] == g[3]) return 0.5;
            return 1.0;
    }
}

/* partners of equal sign listed in ascending global mode index */
static void canonical_order(int ptype, int64_t* g, double* w) {
    int lo, hi;
    if (ptype == T3P) return;
    if (ptype == T3M || ptype == T4PP) { lo = 1; hi = 2; }
    else if (ptype == T4PM) { lo = 2; hi = 3; }
    else { lo = 1; hi = 3; }
    for (int i = lo; i <= hi; ++i)
        for (int j = i + 1; j <= hi; ++j)
            if (g[j] < g[i]) {
                int64_t tg = g[i]; g[i] = g[j]; g[j] = tg;
                double tw = w[i]; w[i] = w[j]; w[j] = tw;
            }
}

/* energy mismatch evaluated left to right in the given partner order */
/*
 * Width of the energy-conservation Gaussian of one process (partners g[1..m-1]).
 * Fixed: sigma.  Adaptive (the per-process width the paper computes from the
 * partners' group velocities, Sec. 3 and Alg. 2-3): the Gaussian whose variance
 * equals that of the mismatch when the free partner wavevectors range uniformly
 * over one mesh cell.  Closing slot k by momentum, the mismatch moves by
 * sum_{r != k} s_r (v_r - v_k).dq_r; a uniform dq over the cell
 * sum_d u_d b_d / N_d (u_d in [-1/2, 1/2]) gives it variance
 * sum_{r != k} sum_d ((v_r - v_k).b_d / N_d)^2 / 12.  Averaged over the choice of
 * k, so that the width is symmetric in the partners, and with sigma^2 = 2 var
 * (the Gaussian exp(-D^2/sigma^2) has variance sigma^2 / 2):
 *   sigma0^2 = sum_{i<j partners} sum_d ((v_i - v_j).b_d / N_d)^2 / (3 (m - 1)),
 * i.e. sum_d ((v' - v'').b_d / N_d)^2 / 6 for three phonons.  Then
 * sigma_p = max(factor * sigma0, sigma).  Pairs (i, j) in ascending slot order,
 * d = 0, 1, 2, each term as written, left to right.
 */
static double process_sigma(const orc_sys* s, int m, const int64_t* g, double sigma) {
    if (!s->adaptive) return sigma;
    double s2 = 0.0;
    for (int i = 1; i < m; ++i)
        for (int j = i + 1; j < m; ++j) {
            const double* vi = s->vel + g[i] * 3;
            const double* vj = s->vel + g[j] * 3;
            double w0 = vi[0] - vj[0], w1 = vi[1] - vj[1], w2 = vi[2] - vj[2];
            for (int d = 0; d < 3; ++d) {
                double p = (w0 * s->recip[d * 3 + 0] + w1 * s->recip[d * 3 + 1] + w2 * s->recip[d * 3 + 2]) /
                           (double)s->mesh[d];
                s2 += p * p;
            }
        }
    double sigma0 = sqrt(s2 / (3.0 * (double)(m - 1)));
    double sp = s->factor * sigma0;
    return sp > sigma ? sp : sigma;
}

static double mismatch(int m, const int32_t* sg, const double* w) {
    double d = w[0];
    for (int r = 1; r < m; ++r) d = sg[r] > 0 ? d + w[r] : d - w[r];
    return d;
}

static double prefactor(int m, int64_t N) {
    double hb = c_hbar();
    if (m == 3) return M_PI * hb / (4.0 * (double)N);
    return M_PI * hb * hb / (8.0 * (double)N * (double)N);
}

static double wp_prefactor(int m, int64_t N) { return m == 3 ? 1.0 / (double)N : 1.0 / ((double)N * (double)N); }

/*
 * One process: partner slots given by integer coordinates and branches.  Adds its
 * Gamma and WP contributions for every temperature.  Returns 1 if it passed the
 * filter (brute mode) or was evaluated (list mode).
 */
typedef struct {
    const orc_sys* s;
    int ptype, m, n_T;
    const double* T;
    double sigma, nsigma;
    int32_t sg[4];
} proc_ctx;

static int process(const proc_ctx* pc, int64_t qc[4][3], const int32_t br[4], double wgt, int filter,
                   ksum* gam, ksum* wp) {
    const orc_sys* s = pc->s;
    int m = pc->m, nb = 3 * s->n_atoms;
    int64_t g[4];
    double w[4];
    for (int r = 0; r < m; ++r) {
        g[r] = q_index(s, qc[r]) * nb + br[r];
        w[r] = s->omega[g[r]];
        if (filter && w[r] < s->omega_floor) return 0;
    }
    int64_t gs[4];
    double ws[4];
    memcpy(gs, g, sizeof g);
    memcpy(ws, w, sizeof w);
    if (filter) canonical_order(pc->ptype, gs, ws);
    double delta = mismatch(m, pc->sg, ws);
    double sp = process_sigma(s, m, gs, pc->sigma);
    if (filter && !(fabs(delta) <= pc->nsigma * sp)) return 0;
    double G = orc_gauss(delta, sp);
    double wprod = 1.0;
    for (int r = 0; r < m; ++r) wprod *= w[r];
    int64_t sq[4][3];
    for (int r = 0; r < m; ++r)
        for (int d = 0; d < 3; ++d) sq[r][d] = qc[r][d];
    cplx V = vertex(s, m, (const int64_t(*)[3])sq, br, pc->sg);
    double V2 = V.re * V.re + V.im * V.im;
    for (int it = 0; it < pc->n_T; ++it) {
        double n[4];
        for (int r = 0; r < m; ++r) n[r] = orc_bose(w[r], pc->T[it]);
        double x = wgt * occupation(pc->ptype, n) * G / wprod;
        kadd(&wp[it], x);
        kadd(&gam[it], x * V2);
    }
    return 1;
}

/* coordinates of the momentum-fixed last slot: q_last = s_last * (-(q + sum of other Q)) */
static void closing_slot(const orc_sys* s, int m, const int32_t* sg, int64_t qc[4][3]) {
    for (int d = 0; d < 3; ++d) {
        int64_t Q = qc[0][d];
        for (int r = 1; r < m - 1; ++r) Q += sg[r] * qc[r][d];
        qc[m - 1][d] = wrap(sg[m - 1] * (-Q), s->mesh[d]);
    }
}

#define MAX_T 16
#define MAX_THREADS 256

/*
 * Per-row rates.  mode 0 = brute (every ordered partner tuple, filter applied),
 * mode 1 = list (records row_off[r]..row_off[r+1] of rec).
 * Outputs (row-major [n_rows][n_T]): gamma (1/ps), wp; n_kept[r] = processes
 * kept (brute) or evaluated (list); n_cand[r] = ordered candidates examined (brute).
 */
int orc_rates(const orc_sys* s, int ptype, int mode, int64_t n_rows, const int32_t* row_mode,
              const int64_t* row_off, const uint64_t* rec, double sigma, double nsigma, int n_T,
              const double* T, double* gamma, double* wp, int64_t* n_kept, int64_t* n_cand) {
    if (ptype < 0 || ptype > 4 || n_T < 1 || n_T > MAX_T) return -1;
    int m = type_order(ptype);
    if ((m == 3 && s->n3 <= 0) || (m == 4 && s->n4 <= 0)) return -2;
    int nb = 3 * s->n_atoms;
    int64_t N = n_q(s);
    proc_ctx pc;
    pc.s = s;
    pc.ptype = ptype;
    pc.m = m;
    pc.n_T = n_T;
    pc.T = T;
    pc.sigma = sigma;
    pc.nsigma = nsigma;
    type_signs(ptype, pc.sg);
    double pre = prefactor(m, N), wpre = wp_prefactor(m, N);
    for (int64_t row = 0; row < n_rows; ++row) {
        int64_t g0 = row_mode[row];
        int64_t q0 = g0 / nb;
        int32_t j0 = (int32_t)(g0 % nb);
        int nthr = 1;
#ifdef _OPENMP
        nthr = omp_get_max_threads();
        if (nthr > MAX_THREADS) nthr = MAX_THREADS;
#endif
        ksum* part = calloc((size_t)nthr * 2 * MAX_T, sizeof(ksum));
        int64_t* kept = calloc((size_t)nthr, sizeof(int64_t));
        int64_t* cand = calloc((size_t)nthr, sizeof(int64_t));
        if (!part || !kept || !cand) {
            free(part); free(kept); free(cand);
            return -3;
        }
        int64_t n_outer = mode == 0 ? N : row_off[row + 1] - row_off[row];
#pragma omp parallel num_threads(nthr)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            ksum* gam = part + (size_t)tid * 2 * MAX_T;
            ksum* wpp = gam + MAX_T;
#pragma omp for schedule(static)
            for (int64_t o = 0; o < n_outer; ++o) {
                int64_t qc[4][3];
                int32_t br[4];
                q_coords(s, q0, qc[0]);
                br[0] = j0;
                if (mode == 0) {
                    /* brute: o is the first partner's q-point */
                    q_coords(s, o, qc[1]);
                    double wgt = ordered_weight(ptype);
                    if (m == 3) {
                        closing_slot(s, 3, pc.sg, qc);
                        for (int j1 = 0; j1 < nb; ++j1)
                            for (int j2 = 0; j2 < nb; ++j2) {
                                br[1] = j1;
                                br[2] = j2;
                                cand[tid]++;
                                kept[tid] += process(&pc, qc, br, wgt, 1, gam, wpp);
                            }
                    } else {
                        for (int64_t q2 = 0; q2 < N; ++q2) {
                            q_coords(s, q2, qc[2]);
                            closing_slot(s, 4, pc.sg, qc);
                            for (int j1 = 0; j1 < nb; ++j1)
                                for (int j2 = 0; j2 < nb; ++j2)
                                    for (int j3 = 0; j3 < nb; ++j3) {
                                        br[1] = j1;
                                        br[2] = j2;
                                        br[3] = j3;
                                        cand[tid]++;
                                        kept[tid] += process(&pc, qc, br, wgt, 1, gam, wpp);
                                    }
                        }
                    }
                } else {
                    /* list: decode the packed record */
                    uint64_t r = rec[row_off[row] + o];
                    int64_t g[4];
                    g[0] = g0;
                    g[1] = (int64_t)(r & 0xFFFFFFu);
                    q_coords(s, g[1] / nb, qc[1]);
                    br[1] = (int32_t)(g[1] % nb);
                    if (m == 3) {
                        br[2] = (int32_t)((r >> 24) & 0xFFu);
                        closing_slot(s, 3, pc.sg, qc);
                    } else {
                        g[2] = (int64_t)((r >> 24) & 0xFFFFFFu);
                        q_coords(s, g[2] / nb, qc[2]);
                        br[2] = (int32_t)(g[2] % nb);
                        br[3] = (int32_t)((r >> 48) & 0xFFu);
                        closing_slot(s, 4, pc.sg, qc);
                    }
                    for (int rr = 1; rr < m; ++rr) g[rr] = q_index(s, qc[rr]) * nb + br[rr];
                    double wgt = triangle_weight(ptype, g);
                    kept[tid] += process(&pc, qc, br, wgt, 0, gam, wpp);
                }
            }
        }
        /* combine per-thread partial sums in thread order */
        for (int it = 0; it < n_T; ++it) {
            ksum tg = {0.0, 0.0}, tw = {0.0, 0.0};
            for (int t = 0; t < nthr; ++t) {
                kadd(&tg, kval(&part[(size_t)t * 2 * MAX_T + it]));
                kadd(&tw, kval(&part[(size_t)t * 2 * MAX_T + MAX_T + it]));
            }
            gamma[row * n_T + it] = pre * kval(&tg);
            wp[row * n_T + it] = wpre * kval(&tw);
        }
        int64_t nk = 0, nc = 0;
        for (int t = 0; t < nthr; ++t) {
            nk += kept[t];
            nc += cand[t];
        }
        if (n_kept) n_kept[row] = nk;
        if (n_cand) n_cand[row] = nc;
        free(part);
        free(kept);
        free(cand);
    }
    return 0;
}

/*
 * Gradient of L = sum_{r,T} dLdG[r][T] * Gamma_r(T) with respect to the raw
 * force-constant entries of the list's order (eV/A^m), added into dphi
 * [n_terms][3^m].  Lists in list mode.  Gamma is quadratic in the force
 * constants:
 *   dL/dPhi_t^{a...} = sum_p c_p 2 Re(conj(V_p) dV_p/dPhi_t^{a...}),
 *   c_p = pref * sum_T dLdG[T] * w occ_T G / prod(omega),
 *   dV_p/dPhi_t^{a...} = eV/sqrt(prod M) eps_0 ... eps_{m-1} exp(i sum Q_r.R_{t,r}).
 */
int orc_grad(const orc_sys* s, int ptype, int64_t n_rows, const int32_t* row_mode, const int64_t* row_off,
             const uint64_t* rec, double sigma, int n_T, const double* T, const double* dLdG, double* dphi) {
    if (ptype < 0 || ptype > 4 || n_T < 1 || n_T > MAX_T) return -1;
    int m = type_order(ptype);
    int64_t n_terms = m == 3 ? s->n3 : s->n4;
    if (n_terms <= 0) return -2;
    const int32_t* atoms = m == 3 ? s->atoms3 : s->atoms4;
    const int32_t* cells = m == 3 ? s->cells3 : s->cells4;
    int ncomp = m == 3 ? 27 : 81;
    int nb = 3 * s->n_atoms;
    int64_t N = n_q(s);
    int32_t sg[4];
    type_signs(ptype, sg);
    double pre = prefactor(m, N), ev = c_ev();
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
    if (nthr > MAX_THREADS) nthr = MAX_THREADS;
#endif
    size_t per = (size_t)n_terms * ncomp;
    ksum* part = calloc((size_t)nthr * per, sizeof(ksum));
    if (!part) return -3;
    int64_t total = row_off[n_rows];
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        ksum* acc = part + (size_t)tid * per;
        int64_t row = 0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < total; ++i) {
            while (row_off[row + 1] <= i) ++row;
            while (row_off[row] > i) --row;
            int64_t qc[4][3] = {{0}};
            int32_t br[4] = {0};
            int64_t g[4] = {0};
            double w[4] = {0.0};
            g[0] = row_mode[row];
            q_coords(s, g[0] / nb, qc[0]);
            br[0] = (int32_t)(g[0] % nb);
            uint64_t r = rec[i];
            g[1] = (int64_t)(r & 0xFFFFFFu);
            q_coords(s, g[1] / nb, qc[1]);
            br[1] = (int32_t)(g[1] % nb);
            if (m == 3) {
                br[2] = (int32_t)((r >> 24) & 0xFFu);
            } else {
                g[2] = (int64_t)((r >> 24) & 0xFFFFFFu);
                q_coords(s, g[2] / nb, qc[2]);
                br[2] = (int32_t)(g[2] % nb);
                br[3] = (int32_t)((r >> 48) & 0xFFu);
            }
            closing_slot(s, m, sg, qc);
            for (int k = 1; k < m; ++k) g[k] = q_index(s, qc[k]) * nb + br[k];
            for (int k = 0; k < m; ++k) w[k] = s->omega[g[k]];
            double delta = mismatch(m, sg, w);
            double G = orc_gauss(delta, process_sigma(s, m, g, sigma));
            double wprod = 1.0;
            for (int k = 0; k < m; ++k) wprod *= w[k];
            double base = triangle_weight(ptype, g) * G / wprod;
            double c = 0.0;
            for (int it = 0; it < n_T; ++it) {
                double n[4];
                for (int k = 0; k < m; ++k) n[k] = orc_bose(w[k], T[it]);
                c += dLdG[row * n_T + it] * pre * base * occupation(ptype, n);
            }
            c *= 2.0;
            cplx V = vertex(s, m, (const int64_t(*)[3])qc, br, sg);
            cplx Vc = {V.re, -V.im};
            for (int64_t t = 0; t < n_terms; ++t) {
                const int32_t* at = atoms + t * m;
                const int32_t* ce = cells + t * (m - 1) * 3;
                int64_t k3[3] = {0, 0, 0};
                for (int rr = 1; rr < m; ++rr)
                    for (int d = 0; d < 3; ++d) k3[d] += (int64_t)sg[rr] * qc[rr][d] * ce[(rr - 1) * 3 + d];
                cplx ph = root_of_unity(s, k3);
                double msc = 1.0;
                for (int rr = 0; rr < m; ++rr) msc *= s->masses[at[rr]];
                cplx f = cmul(Vc, ph);
                double sc = c * ev / sqrt(msc);
                for (int idx = 0; idx < ncomp; ++idx) {
                    int a[4];
                    int rem = idx;
                    for (int rr = m - 1; rr >= 0; --rr) {
                        a[rr] = rem % 3;
                        rem /= 3;
                    }
                    cplx prod = f;
                    for (int rr = 0; rr < m; ++rr) prod = cmul(prod, evec_at(s, g[rr], 3 * at[rr] + a[rr], sg[rr]));
                    kadd(&acc[t * ncomp + idx], sc * prod.re);
                }
            }
        }
    }
    for (size_t k = 0; k < per; ++k) {
        ksum tot = {0.0, 0.0};
        for (int t = 0; t < nthr; ++t) kadd(&tot, kval(&part[(size_t)t * per + k]));
        dphi[k] += kval(&tot);
    }
    free(part);
    return 0;
}

/*
 * Brute-force enumeration of one row: every ordered partner tuple that passes the
 * filter and whose equal-sign partners are already in ascending mode order is
 * written as a packed record (3ph: g1 | j2<<24; 4ph: g1 | g2<<24 | j3<<48).
 * Returns the number of such records (only the first `cap` are written).
 */
int64_t orc_enumerate(const orc_sys* s, int ptype, int32_t row_mode, double sigma, double nsigma, uint64_t* out,
                      int64_t cap) {
    int m = type_order(ptype);
    int nb = 3 * s->n_atoms;
    int64_t N = n_q(s);
    int32_t sg[4];
    type_signs(ptype, sg);
    int64_t count = 0;
    int64_t qc[4][3];
    int32_t br[4];
    q_coords(s, row_mode / nb, qc[0]);
    br[0] = row_mode % nb;
    if (s->omega[row_mode] < s->omega_floor) return 0;
    int64_t n2 = m == 3 ? 1 : N;
    for (int64_t q1 = 0; q1 < N; ++q1) {
        q_coords(s, q1, qc[1]);
        for (int64_t q2 = 0; q2 < n2; ++q2) {
            if (m == 4) q_coords(s, q2, qc[2]);
            closing_slot(s, m, sg, qc);
            int nbr = m == 3 ? nb * nb : nb * nb * nb;
            for (int b = 0; b < nbr; ++b) {
                br[1] = b / (m == 3 ? nb : nb * nb);
                br[2] = m == 3 ? b % nb : (b / nb) % nb;
                if (m == 4) br[3] = b % nb;
                int64_t g[4];
                double w[4];
                int ok = 1;
                for (int r = 0; r < m; ++r) {
                    g[r] = q_index(s, qc[r]) * nb + br[r];
                    w[r] = s->omega[g[r]];
                    if (w[r] < s->omega_floor) ok = 0;
                }
                if (!ok) continue;
                int64_t gs[4];
                double ws[4];
                memcpy(gs, g, sizeof g);
                memcpy(ws, w, sizeof w);
                canonical_order(ptype, gs, ws);
                if (memcmp(gs, g, sizeof(int64_t) * m) != 0) continue; /* not the canonical ordering */
                double delta = mismatch(m, sg, ws);
                if (!(fabs(delta) <= nsigma * process_sigma(s, m, gs, sigma))) continue;
                uint64_t r = (uint64_t)g[1];
                if (m == 3)
                    r |= (uint64_t)br[2] << 24;
                else
                    r |= ((uint64_t)g[2] << 24) | ((uint64_t)br[3] << 48);
                if (count < cap) out[count] = r;
                count++;
            }
        }
    }
    return count;
}

/*
 * kappa^{ab} = 1/(N Omega kB T^2) sum_{q in Q1} w_q sum_j n(n+1) (hbar w)^2 v^a v^b / Gamma,
 * in W/(m K).  Modes with omega < floor or Gamma <= 0 contribute nothing.
 * gamma is indexed by global mode g.
 */
int orc_kappa(int32_t nq1, const int32_t* q1, const double* q1_weight, int32_t nb, const double* omega,
              const double* vel, const double* gamma, double T, double volume, int64_t N, double omega_floor,
              double* kappa) {
    double hb = c_hbar(), kb = c_kb();
    ksum acc[9];
    memset(acc, 0, sizeof acc);
    for (int32_t i = 0; i < nq1; ++i)
        for (int32_t j = 0; j < nb; ++j) {
            int64_t g = (int64_t)q1[i] * nb + j;
            double w = omega[g];
            if (w < omega_floor || !(gamma[g] > 0.0)) continue;
            double n = orc_bose(w, T);
            double c = q1_weight[i] * n * (n + 1.0) * (hb * w) * (hb * w) / gamma[g];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) kadd(&acc[a * 3 + b], c * vel[g * 3 + a] * vel[g * 3 + b]);
        }
    double pre = c_kappa() / ((double)N * volume * kb * T * T);
    for (int k = 0; k < 9; ++k) kappa[k] = pre * kval(&acc[k]);
    return 0;
}
