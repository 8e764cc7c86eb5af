// Host enumeration of filtered, triangle-reduced process lists (the CPU half of
// the paper's hybrid scheme, Appendix Algorithm 3, generalised to both
// three-phonon signs and the three four-phonon types).
//
// Pass 1 counts the kept partners of every row (the paper's N_plus) and forms
// their exclusive prefix sum (N_accum); pass 2 writes the packed records
// (Ind2/Ind3).  Rows are distributed over std::threads with an atomic counter;
// each row is written by exactly one thread, so the output does not depend on
// the thread count.
//
// The energy mismatch is evaluated in double precision, strictly left to right
// in record order, and this file is compiled without floating-point
// contraction, so the filter decision is reproducible bit for bit.  So is the
// adaptive width: the partner pairs in record order, the three reciprocal
// directions in order, each projection ((v_i - v_j) . b_d) / N_d as written.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "fp.h"
#include "fp_enum_impl.h"

#pragma clang fp contract(off)

namespace {

struct TypeInfo {
    int order;
    int s[4];  // signs of slots 0..order-1 (slot 0 is the mode itself, +1)
};

bool type_info(int32_t type, TypeInfo* ti) {
    switch (type) {
        case FP_3P: *ti = {3, {1, 1, -1, 0}}; return true;
        case FP_3M: *ti = {3, {1, -1, -1, 0}}; return true;
        case FP_4PP: *ti = {4, {1, 1, 1, -1}}; return true;
        case FP_4PM: *ti = {4, {1, 1, -1, -1}}; return true;
        case FP_4MM: *ti = {4, {1, -1, -1, -1}}; return true;
        case FP_3E: *ti = {3, {1, 1, -1, 0}}; return true;  // events lambda + lambda' -> lambda''
        default: return false;
    }
}

inline int64_t wrapi(int64_t x, int64_t n) { return ((x % n) + n) % n; }

// SplitMix64 finaliser (Steele, Lea, Flood 2014): the hash behind keep_fraction.
inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct Enum {
    TypeInfo ti;
    bool events;  // FP_3E
    int64_t N[3], nq;
    int32_t nb;
    const double* omega;
    double floor_, cut;
    uint64_t keep_threshold;  // keep iff hash < threshold (all when keep_all)
    bool keep_all;
    uint64_t seed;
    // adaptive broadening: sigma_p = max(factor * sigma0_p, sigma); cut_max bounds
    // nsigma * sigma_p over every process, so a candidate beyond it is rejected
    // without evaluating its width
    bool adaptive;
    const double* vel;
    double recip[9], factor, sigma, nsigma, cut_max;
    // frequency bounds (order 4): per q-point the smallest and largest branch
    // frequency, and over the mesh the smallest active and the largest one
    std::vector<double> wlo, whi;
    double wmin_act = 0.0, wmax_all = 0.0;
    // adaptive width, order 4: per q-point the largest |v_g . b_d / N_d| over its
    // branches, so that a (q', q'', q''') triple bounds its processes' widths;
    // per mode the projections (v_g . b_d) * (1 / N_d), whose pair differences
    // give the width to within perr, so the filter's own arithmetic is needed
    // only where |Delta| falls inside that bracket
    std::vector<double> pq, proj;
    double perr = 0.0;

    // squared projections of one partner pair, summed over the three directions
    // into s2 in order
    double pair_sq(double s2, int64_t gi, int64_t gj) const {
        const double* vi = vel + gi * 3;
        const double* vj = vel + gj * 3;
        const double w0 = vi[0] - vj[0], w1 = vi[1] - vj[1], w2 = vi[2] - vj[2];
        for (int d = 0; d < 3; ++d) {
            const double p = (w0 * recip[d * 3 + 0] + w1 * recip[d * 3 + 1] + w2 * recip[d * 3 + 2]) / (double)N[d];
            s2 += p * p;
        }
        return s2;
    }
    // the filter: |delta| <= nsigma * sigma_p; s2 holds the pairs not involving
    // the last partner (summed first, as their slots come first).  The fixed
    // cut decides most candidates, so it stays inline and the width test apart.
    __attribute__((always_inline)) bool pass(double delta, double cut_fixed, double cut_lim, int m, double s2_head,
                                             int64_t gl_prev0, int64_t gl_prev1, int64_t gl) const {
        const double ad = std::fabs(delta);
        if (ad <= cut_fixed) return true;   // sigma_p >= sigma
        if (!adaptive || !(ad <= cut_lim)) return false;
        return pass_width(ad, m, s2_head, gl_prev0, gl_prev1, gl);
    }
    bool pass_width(double ad, int m, double s2_head, int64_t gl_prev0, int64_t gl_prev1, int64_t gl) const {
        if (m == 4) {
            // the norm of the nine pair projections lies within
            // [n (1 - rel) - perr, n (1 + rel) + perr] of the table's n; the
            // outer factors cover the rounding of the width formula itself
            const double *p1 = &proj[(size_t)gl_prev0 * 3], *p2 = &proj[(size_t)gl_prev1 * 3],
                         *p3 = &proj[(size_t)gl * 3];
            const double* pp[3][2] = {{p1, p2}, {p1, p3}, {p2, p3}};
            double t2 = 0.0;  // pairs in slot order, directions inside
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 3; ++d) {
                    const double t = pp[k][0][d] - pp[k][1][d];
                    t2 += t * t;
                }
            const double nrm = std::sqrt(t2);
            constexpr double rel = 1e-13;
            const double sp_lo = factor / 3.0 * (nrm * (1.0 - rel) - perr) * (1.0 - rel);
            const double sp_hi = factor / 3.0 * (nrm * (1.0 + rel) + perr) * (1.0 + rel);
            if (ad <= nsigma * std::max(sp_lo, sigma) * (1.0 - rel)) return true;
            if (ad > nsigma * std::max(sp_hi, sigma) * (1.0 + rel)) return false;
            s2_head = pair_sq(0.0, gl_prev0, gl_prev1);
        }
        double s2 = pair_sq(s2_head, gl_prev0, gl);
        if (m == 4) s2 = pair_sq(s2, gl_prev1, gl);
        const double sp = factor * std::sqrt(s2 / (3.0 * (double)(m - 1)));
        return ad <= nsigma * (sp > sigma ? sp : sigma);
    }

    void coords(int64_t iq, int64_t c[3]) const {
        c[2] = iq % N[2];
        c[1] = (iq / N[2]) % N[1];
        c[0] = iq / (N[1] * N[2]);
    }
    int64_t index(const int64_t c[3]) const {
        return (wrapi(c[0], N[0]) * N[1] + wrapi(c[1], N[1])) * N[2] + wrapi(c[2], N[2]);
    }
    // keep_fraction samples whole (q', q'') pairs (3ph: q'), so a subsampled list
    // holds every branch combination of the pairs it keeps, like a full list
    bool keep(uint64_t row_g, uint64_t iq1, uint64_t iq2) const {
        if (keep_all) return true;
        return mix64(seed ^ mix64(row_g ^ mix64((iq1 << 32) | iq2))) < keep_threshold;
    }

    // The largest nsigma * sigma_p of any branch triple of three q-points: each
    // pair's projection difference is at most the sum of the two maxima, and the
    // relative margin lies far above the rounding of either evaluation.
    double cut_bound(int64_t iq1, int64_t iq2, int64_t iq3) const {
        const double *p1 = &pq[(size_t)iq1 * 3], *p2 = &pq[(size_t)iq2 * 3], *p3 = &pq[(size_t)iq3 * 3];
        double b2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double a = p1[d] + p2[d], b = p1[d] + p3[d], c = p2[d] + p3[d];
            b2 += a * a + b * b + c * c;
        }
        const double sp = std::max(factor * std::sqrt(b2 / 9.0), sigma);
        return std::min(nsigma * sp * (1.0 + 1e-9), cut_max);
    }

    // Visit the kept records of row mode g0 in (q', q'', j', j'', j''') order (3ph: q', j', j'').
    template <class F>
    void row(int64_t g0, F&& emit) const {
        const double w0 = omega[g0];
        if (!(w0 >= floor_)) return;
        int64_t q0[3];
        coords(g0 / nb, q0);
        const int* s = ti.s;
        if (ti.order == 3) {
            for (int64_t iq1 = 0; iq1 < nq; ++iq1) {
                if (!keep((uint64_t)g0, (uint64_t)iq1, 0)) continue;
                int64_t q1[3], q2[3];
                coords(iq1, q1);
                // s2 q2 = -(q0 + s1 q1)
                for (int d = 0; d < 3; ++d) q2[d] = s[2] * (-(q0[d] + s[1] * q1[d]));
                const int64_t iq2 = index(q2);
                for (int32_t j1 = 0; j1 < nb; ++j1) {
                    const int64_t g1 = iq1 * nb + j1;
                    if (events && g1 < g0) continue;  // FP_3E: g' >= g, one record per event
                    const double w1 = omega[g1];
                    if (!(w1 >= floor_)) continue;
                    const double d1 = s[1] > 0 ? w0 + w1 : w0 - w1;
                    for (int32_t j2 = 0; j2 < nb; ++j2) {
                        const int64_t g2 = iq2 * nb + j2;
                        if (ti.s[1] < 0 && g2 < g1) continue;  // FP_3M: g' <= g''
                        const double w2 = omega[g2];
                        if (!(w2 >= floor_)) continue;
                        const double delta = s[2] > 0 ? d1 + w2 : d1 - w2;
                        if (events) {
                            // the 3+ processes of g and g' (mismatch as in their FP_3P
                            // lists) and the 3- process of g'' (as in its FP_3M list,
                            // partners g <= g')
                            const bool plus = std::fabs(delta) <= cut;
                            const bool minus = std::fabs((w2 - w0) - w1) <= cut;
                            if (!plus && !minus) continue;
                            emit((uint64_t)g1 | ((uint64_t)j2 << 24) | ((uint64_t)plus << 32) |
                                 ((uint64_t)minus << 33));
                            continue;
                        }
                        if (!pass(delta, cut, cut_max, 3, 0.0, g1, 0, g2)) continue;
                        emit((uint64_t)g1 | ((uint64_t)j2 << 24));
                    }
                }
            }
            return;
        }
        const bool tri12 = (s[1] == s[2]);            // ++ and --: g' <= g''
        const bool tri23 = (s[2] == s[3]);            // +- and --: g'' <= g'''
        // Frequency bounds skip blocks of candidates that cannot pass: with the
        // partners' frequencies between their q-point's (or the mesh's) extremes,
        // every mismatch of a block lies in an interval (sums in the filter's
        // order; rounding is monotone, and a 1e-9 relative margin is added), and
        // a block whose interval misses the widest cut holds no kept record.  The
        // decisions and the order of the kept records are the filter's own.
        const double cut_any = adaptive ? cut_max : cut;
        // q''' per axis as a function of q'' (s3 q''' = -(q + s1 q' + s2 q'')),
        // tabulated once per q', with q'' stepped through the mesh in index order:
        // no integer division per q-point pair
        std::vector<int64_t> t3((size_t)(N[0] + N[1] + N[2]));
        int64_t* const t30 = t3.data();
        int64_t* const t31 = t30 + N[0];
        int64_t* const t32 = t31 + N[1];
        // per mode the signed frequencies of slots 2 and 3 (a - b is a + (-b), so
        // the mismatch keeps its bits), NaN below the floor: a NaN mismatch fails
        // every cut, so the floor test leaves the innermost loop
        const int64_t nm = nq * nb;
        std::vector<double> sw((size_t)nm * 2);
        double* const sw2 = sw.data();
        double* const sw3 = sw2 + nm;
        for (int64_t g = 0; g < nm; ++g) {
            const double w = omega[g];
            const bool act = w >= floor_;
            sw2[g] = act ? (s[2] > 0 ? w : -w) : NAN;
            sw3[g] = act ? (s[3] > 0 ? w : -w) : NAN;
        }
        auto step = [&](int64_t* c) {
            if (++c[2] == N[2]) {
                c[2] = 0;
                if (++c[1] == N[1]) {
                    c[1] = 0;
                    ++c[0];
                }
            }
        };
        // q-point pairs outermost, so the records of one (q', q'') tuple are contiguous
        for (int64_t iq1 = 0; iq1 < nq; ++iq1) {
            {
                const double w1l = wlo[(size_t)iq1], w1h = whi[(size_t)iq1];
                double lo = s[1] > 0 ? w0 + w1l : w0 - w1h;
                lo = s[2] > 0 ? lo + wmin_act : lo - wmax_all;
                lo = s[3] > 0 ? lo + wmin_act : lo - wmax_all;
                double hi = s[1] > 0 ? w0 + w1h : w0 - w1l;
                hi = s[2] > 0 ? hi + wmax_all : hi - wmin_act;
                hi = s[3] > 0 ? hi + wmax_all : hi - wmin_act;
                const double cu = cut_any + 1e-9 * (w0 + w1h + 2.0 * wmax_all);
                if (lo > cu || hi < -cu) continue;
            }
            int64_t q1[3];
            coords(iq1, q1);
            int64_t* const tt[3] = {t30, t31, t32};
            for (int d = 0; d < 3; ++d)
                for (int64_t x = 0; x < N[d]; ++x) tt[d][x] = wrapi(s[3] * (-(q0[d] + s[1] * q1[d] + s[2] * x)), N[d]);
            const int64_t iq2_0 = tri12 ? iq1 : 0;
            int64_t q2[3];
            coords(iq2_0, q2);
            for (int64_t iq2 = iq2_0; iq2 < nq; ++iq2, step(q2)) {
                if (!keep((uint64_t)g0, (uint64_t)iq1, (uint64_t)iq2)) continue;
                const int64_t iq3 = (t30[q2[0]] * N[1] + t31[q2[1]]) * N[2] + t32[q2[2]];
                if (tri23 && iq3 < iq2) continue;  // every g''' < g'': the triangle keeps none
                const double lo2 = s[2] > 0 ? wlo[(size_t)iq2] : -whi[(size_t)iq2];
                const double hi2 = s[2] > 0 ? whi[(size_t)iq2] : -wlo[(size_t)iq2];
                const double lo3 = s[3] > 0 ? wlo[(size_t)iq3] : -whi[(size_t)iq3];
                const double hi3 = s[3] > 0 ? whi[(size_t)iq3] : -wlo[(size_t)iq3];
                // the widest cut of this q-point triple (adaptive: its width bound)
                const double cut_q = adaptive ? cut_bound(iq1, iq2, iq3) : cut;
                const double cmax = cut_q + 1e-9 * (w0 + whi[(size_t)iq1] + whi[(size_t)iq2] + whi[(size_t)iq3]);
                for (int32_t j1 = 0; j1 < nb; ++j1) {
                    const int64_t g1 = iq1 * nb + j1;
                    const double w1 = omega[g1];
                    if (!(w1 >= floor_)) continue;
                    const double d1 = s[1] > 0 ? w0 + w1 : w0 - w1;
                    if (d1 + lo2 + lo3 > cmax || d1 + hi2 + hi3 < -cmax) continue;
                    for (int32_t j2 = 0; j2 < nb; ++j2) {
                        const int64_t g2 = iq2 * nb + j2;
                        if (tri12 && g2 < g1) continue;
                        const double d2 = d1 + sw2[g2];
                        if (!(d2 + lo3 <= cmax && d2 + hi3 >= -cmax)) continue;  // NaN: inactive
                        for (int32_t j3 = tri23 && iq3 == iq2 ? j2 : 0; j3 < nb; ++j3) {
                            const int64_t g3 = iq3 * nb + j3;
                            if (tri23 && g3 < g2) continue;
                            const double delta = d2 + sw3[g3];
                            if (!pass(delta, cut, cut_q, 4, 0.0, g1, g2, g3)) continue;
                            emit((uint64_t)g1 | ((uint64_t)g2 << 24) | ((uint64_t)j3 << 48));
                        }
                    }
                }
            }
        }
    }
};

fp_status setup(Enum* e, int32_t type, const int32_t mesh[3], int32_t nb, const double* omega, double omega_floor,
                int64_t n_rows, const int32_t* row_mode, double sigma, double nsigma, double keep_fraction,
                uint64_t seed, const double* vel, const fp_broadening* br) {
    if (!mesh || !omega || (n_rows > 0 && !row_mode) || n_rows < 0) return FP_ERR_ARG;
    if (!type_info(type, &e->ti)) return FP_ERR_ARG;
    if (nb < 1 || nb > 96 || !(sigma > 0.0) || !(nsigma > 0.0) || !(keep_fraction > 0.0 && keep_fraction <= 1.0))
        return FP_ERR_ARG;
    e->nq = 1;
    for (int d = 0; d < 3; ++d) {
        if (mesh[d] < 1) return FP_ERR_ARG;
        e->N[d] = mesh[d];
        e->nq *= mesh[d];
    }
    if (e->nq * nb >= (int64_t(1) << 24)) return FP_ERR_UNSUPPORTED;
    for (int64_t r = 0; r < n_rows; ++r)
        if (row_mode[r] < 0 || row_mode[r] >= e->nq * nb) return FP_ERR_ARG;
    e->nb = nb;
    e->omega = omega;
    e->floor_ = omega_floor;
    e->cut = nsigma * sigma;
    if (e->ti.order == 4) {
        e->wlo.assign((size_t)e->nq, 0.0);
        e->whi.assign((size_t)e->nq, 0.0);
        e->wmin_act = HUGE_VAL;
        e->wmax_all = 0.0;
        for (int64_t q = 0; q < e->nq; ++q) {
            double lo = omega[q * nb], hi = omega[q * nb];
            for (int32_t j = 0; j < nb; ++j) {
                const double w = omega[q * nb + j];
                lo = std::min(lo, w);
                hi = std::max(hi, w);
                if (w >= omega_floor) e->wmin_act = std::min(e->wmin_act, w);
            }
            e->wlo[(size_t)q] = lo;
            e->whi[(size_t)q] = hi;
            e->wmax_all = std::max(e->wmax_all, hi);
        }
    }
    e->keep_all = keep_fraction >= 1.0;
    e->keep_threshold = e->keep_all ? ~0ULL : (uint64_t)std::ldexp(keep_fraction, 64);
    e->seed = seed;
    e->events = type == FP_3E;
    e->adaptive = br && br->adaptive;
    if (e->events && e->adaptive) return FP_ERR_UNSUPPORTED;
    e->sigma = sigma;
    e->nsigma = nsigma;
    e->vel = vel;
    e->factor = 0.0;
    e->cut_max = e->cut;
    if (br && br->adaptive != 0 && br->adaptive != 1) return FP_ERR_ARG;
    if (e->adaptive) {
        if (!vel || !(br->factor > 0.0) || !std::isfinite(br->factor)) return FP_ERR_ARG;
        for (int i = 0; i < 9; ++i) {
            if (!std::isfinite(br->recip[i])) return FP_ERR_ARG;
            e->recip[i] = br->recip[i];
        }
        e->factor = br->factor;
        // bound: |(v_i - v_j).b_d / N_d| <= 2 max_g |v_g . b_d| / N_d for every pair
        double pmax[3] = {0.0, 0.0, 0.0};
        const int64_t nm = e->nq * nb;
        for (int64_t g = 0; g < nm; ++g) {
            for (int i = 0; i < 3; ++i)
                if (!std::isfinite(vel[g * 3 + i])) return FP_ERR_ARG;
            for (int d = 0; d < 3; ++d) {
                const double p = std::fabs(vel[g * 3] * e->recip[d * 3] + vel[g * 3 + 1] * e->recip[d * 3 + 1] +
                                           vel[g * 3 + 2] * e->recip[d * 3 + 2]) /
                                 (double)e->N[d];
                if (p > pmax[d]) pmax[d] = p;
            }
        }
        const int m = e->ti.order;
        const double n_pairs = m == 3 ? 1.0 : 3.0;
        double b2 = 0.0;
        for (int d = 0; d < 3; ++d) b2 += 4.0 * pmax[d] * pmax[d];
        const double smax = std::max(e->factor * std::sqrt(n_pairs * b2 / (3.0 * (double)(m - 1))), sigma);
        // relative margin far above the rounding of either evaluation
        e->cut_max = nsigma * smax * (1.0 + 1e-9);
        if (m == 4) {
            e->pq.assign((size_t)e->nq * 3, 0.0);
            e->proj.assign((size_t)nm * 3, 0.0);
            double babs = 0.0;  // max over modes and directions of sum_k |v_k b_dk| / N_d
            for (int64_t g = 0; g < nm; ++g)
                for (int d = 0; d < 3; ++d) {
                    const double* v = vel + g * 3;
                    const double* b = e->recip + d * 3;
                    const double p = std::fabs(v[0] * b[0] + v[1] * b[1] + v[2] * b[2]) / (double)e->N[d];
                    double& x = e->pq[(size_t)(g / nb) * 3 + d];
                    if (p > x) x = p;
                    e->proj[(size_t)g * 3 + d] = (v[0] * b[0] + v[1] * b[1] + v[2] * b[2]) * (1.0 / (double)e->N[d]);
                    babs = std::max(babs, (std::fabs(v[0] * b[0]) + std::fabs(v[1] * b[1]) + std::fabs(v[2] * b[2])) /
                                              (double)e->N[d]);
                }
            e->perr = 3e-12 * babs;
        }
    }
    return FP_OK;
}

template <class F>
void parallel_rows(int64_t n_rows, int32_t n_threads, F&& body) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = n_threads > 0 ? n_threads : (hw ? hw : 1);
    if (nt > n_rows) nt = n_rows > 0 ? n_rows : 1;
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        for (;;) {
            int64_t r = next.fetch_add(1);
            if (r >= n_rows) break;
            body(r);
        }
    };
    std::vector<std::thread> pool;
    for (int64_t t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
}

}  // namespace

extern "C" fp_status fp_enumerate_count(int32_t type, const int32_t mesh[3], int32_t nb, const double* omega,
                                        double omega_floor, int64_t n_rows, const int32_t* row_mode, double sigma,
                                        double nsigma, double keep_fraction, uint64_t seed, int32_t n_threads,
                                        const double* vel, const fp_broadening* broadening, int64_t* row_off) {
    Enum e;
    fp_status st = setup(&e, type, mesh, nb, omega, omega_floor, n_rows, row_mode, sigma, nsigma, keep_fraction,
                         seed, vel, broadening);
    if (st != FP_OK) return st;
    if (!row_off) return FP_ERR_ARG;
    std::vector<int64_t> cnt((size_t)n_rows, 0);
    parallel_rows(n_rows, n_threads, [&](int64_t r) {
        int64_t c = 0;
        e.row(row_mode[r], [&](uint64_t) { ++c; });
        cnt[(size_t)r] = c;
    });
    row_off[0] = 0;
    for (int64_t r = 0; r < n_rows; ++r) row_off[r + 1] = row_off[r] + cnt[(size_t)r];
    return FP_OK;
}

extern "C" fp_status fp_enumerate_fill(int32_t type, const int32_t mesh[3], int32_t nb, const double* omega,
                                       double omega_floor, int64_t n_rows, const int32_t* row_mode, double sigma,
                                       double nsigma, double keep_fraction, uint64_t seed, int32_t n_threads,
                                       const double* vel, const fp_broadening* broadening, const int64_t* row_off,
                                       uint64_t* rec) {
    Enum e;
    fp_status st = setup(&e, type, mesh, nb, omega, omega_floor, n_rows, row_mode, sigma, nsigma, keep_fraction,
                         seed, vel, broadening);
    if (st != FP_OK) return st;
    if (!row_off || (!rec && row_off[n_rows] > 0)) return FP_ERR_ARG;
    std::atomic<int> bad(0);
    parallel_rows(n_rows, n_threads, [&](int64_t r) {
        int64_t pos = row_off[r];
        const int64_t end = row_off[r + 1];
        e.row(row_mode[r], [&](uint64_t v) {
            if (pos < end) rec[pos] = v;
            ++pos;
        });
        if (pos != end) bad.store(1);
    });
    return bad.load() ? FP_ERR_ARG : FP_OK;
}

// ------------------------------------------------ streaming executor interface

namespace fpenum {

struct Handle {
    Enum e;
};

fp_status open(Handle** h, int32_t type, const int32_t mesh[3], int32_t nb, const double* omega,
               double omega_floor, double sigma, double nsigma, const double* vel, const fp_broadening* br) {
    if (!h) return FP_ERR_ARG;
    *h = nullptr;
    Handle* p = new (std::nothrow) Handle;
    if (!p) return FP_ERR_NOMEM;
    fp_status st = setup(&p->e, type, mesh, nb, omega, omega_floor, 0, nullptr, sigma, nsigma, 1.0, 0, vel, br);
    if (st != FP_OK) {
        delete p;
        return st;
    }
    *h = p;
    return FP_OK;
}

void close(Handle* h) { delete h; }

int64_t count_row(const Handle* h, int32_t g0) {
    int64_t c = 0;
    h->e.row(g0, [&](uint64_t) { ++c; });
    return c;
}

int64_t fill_row(const Handle* h, int32_t g0, int64_t begin, int64_t end, uint64_t* out) {
    int64_t i = 0, n = 0;
    h->e.row(g0, [&](uint64_t v) {
        if (i >= begin && i < end) {
            out[i - begin] = v;
            ++n;
        }
        ++i;
    });
    return n;
}

void parallel_for(int64_t n, int32_t n_threads, const std::function<void(int64_t)>& body) {
    parallel_rows(n, n_threads, body);
}

}  // namespace fpenum
