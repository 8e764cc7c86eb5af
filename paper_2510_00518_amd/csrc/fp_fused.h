// Four-phonon rates with the process lists generated on the GPU.
// Included once, by fp_lib.hip, after fp_batched.h.
//
// The host enumerator (Appendix, Algorithm 3) walks every (q', q'') pair of a
// row and keeps the branch triples that pass the energy filter; at a 16^3 mesh
// its lists no longer fit in memory.  Here the walk runs on the GPU and feeds
// the tuple-batched evaluation directly, so no list is ever stored:
//   - a work unit is (type, row lambda, q'); a wave takes 64 values of q'' at a
//     time, one per lane, and closes q''' by momentum;
//   - each lane tests its nb^3 branch triples with exactly the host's rules
//     (FP64 mismatch left to right, no contraction, "<=", frequency floor,
//     triangle order on the global mode index) into a bit mask;
//   - a wave-wide prefix sum of the mask popcounts orders the kept records by
//     (q'', j', j'', j''') -- the enumerator's order -- and the records are
//     decoded from the masks (binary search over the prefix, select the n-th
//     set bit; masks and prefixes are read across lanes by shuffles, so the
//     kernel needs no more LDS than the list-driven one) into a 128-record
//     buffer that fills across chunks of q'' and is evaluated by tb_batch (or
//     tbm_batch) when full and at the end of the unit;
//   - each XCD takes one slice of the q' range of every row;
//   - the rates of a unit go to one partial per unit, summed per row by
//     k_finalize in unit order; the unit's kept processes and tuples go to
//     per-unit counters.
// Compiled for nb = 6 (two-atom cells): the 216 candidate bits of a lane are
// then compile-time positions in four 64-bit registers.
#pragma once

namespace fpk {

constexpr int kFusedNb = 6;
// FP64 instantiations: 24-tuple batches and three resident blocks per CU (16^3
// cell 16.5 s against 19.4 s at 32 and two); the mixed ones keep 32 and two,
// which measured faster for them
constexpr int kFusedTB = 24;

struct FusedArgs {
    int64_t n_units;  // n_types * n_rows * Nq
    int64_t n_rows;
    int32_t n_types;
    int32_t types[3];
    double floor_, cut;
    // adaptive width (the ADAPT instantiation): sigma_p = max(factor sigma0_p,
    // sigma); a candidate with cut < |Delta| <= cut_max has its width evaluated
    // exactly as the host enumerator does
    const double* vel;
    double recip[9];
    double factor, sigma, nsigma, cut_max;
    // bound on |norm of the nine pair projections from the per-mode table P
    // minus the same norm in the enumerator's arithmetic| (3e-12 max_g,d
    // sum_k |v_gk b_dk| / N_d: several hundred times the rounding of either)
    double perr;
};

// |Delta| <= nsigma * sigma_p for partners g1, g2, g3 of a four-phonon process,
// evaluated as the host enumerator evaluates it: pairs (1,2), (1,3), (2,3),
// each projection ((v_i - v_j) . b_d) / N_d, d = 0, 1, 2, summed left to right
// in double precision without contraction; correctly rounded square root and
// division.
__device__ inline double fused_pair_sq(double s2, const double* __restrict__ vel, int32_t gi, int32_t gj,
                                       const FusedArgs& f, const ModeGeom& geo) {
#pragma clang fp contract(off)
    const double w0 = vel[gi * 3] - vel[gj * 3];
    const double w1 = vel[gi * 3 + 1] - vel[gj * 3 + 1];
    const double w2 = vel[gi * 3 + 2] - vel[gj * 3 + 2];
    const double n[3] = {(double)geo.N0, (double)geo.N1, (double)geo.N2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double p = (w0 * f.recip[d * 3] + w1 * f.recip[d * 3 + 1] + w2 * f.recip[d * 3 + 2]) / n[d];
        s2 = s2 + p * p;
    }
    return s2;
}

// max over the branches of one q-point of |v . b_d| / N_d, d = 0, 1, 2: bounds
// the pair projections of the adaptive width from above
__device__ inline void fused_proj_max(const double* __restrict__ vel, int32_t iq, const FusedArgs& f,
                                      const ModeGeom& geo, double (&pm)[3]) {
    const double n[3] = {(double)geo.N0, (double)geo.N1, (double)geo.N2};
    pm[0] = pm[1] = pm[2] = 0.0;
#pragma unroll
    for (int j = 0; j < kFusedNb; ++j) {
        const double* v = vel + ((int64_t)iq * kFusedNb + j) * 3;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            pm[d] = fmax(pm[d], fabs(v[0] * f.recip[d * 3] + v[1] * f.recip[d * 3 + 1] + v[2] * f.recip[d * 3 + 2]) / n[d]);
    }
}

// Largest nsigma * sigma_p any branch triple of the q-points with projection
// bounds p1, p2, p3 can reach (with a margin far above rounding).
__device__ inline double fused_cut_bound(const double (&p1)[3], const double (&p2)[3], const double (&p3)[3],
                                         const FusedArgs& f) {
    double b2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double a = p1[d] + p2[d], b = p1[d] + p3[d], c = p2[d] + p3[d];
        b2 += a * a + b * b + c * c;
    }
    const double sp = fmax(f.factor * sqrt(b2 / 9.0), f.sigma);
    return fmin(f.nsigma * sp * (1.0 + 1e-9), f.cut_max);
}

// not inlined: the exact width is needed only for the few candidates between
// the two cuts, which each lane walks after its unrolled filter loop
__device__ __noinline__ bool fused_adaptive_pass(double ad, int32_t g1, int32_t g2, int32_t g3, const FusedArgs& f,
                                           const ModeGeom& geo) {
#pragma clang fp contract(off)
    double s2 = fused_pair_sq(0.0, f.vel, g1, g2, f, geo);
    s2 = fused_pair_sq(s2, f.vel, g1, g3, f, geo);
    s2 = fused_pair_sq(s2, f.vel, g2, g3, f, geo);
    const double sp = f.factor * __builtin_sqrt(s2 / 9.0);
    return ad <= f.nsigma * (sp > f.sigma ? sp : f.sigma);
}

// Row and unit tables of a fused call: fused row fr = ti * n_rows + r.
__global__ void k_fused_rows(const int32_t* __restrict__ row_mode, FusedArgs f, int64_t nq, int64_t n_modes,
                             RowInfo* __restrict__ rows, int64_t* __restrict__ unit_off, int* flag) {
    const int64_t n = (int64_t)f.n_types * f.n_rows;
    for (int64_t fr = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; fr <= n; fr += (int64_t)gridDim.x * blockDim.x) {
        unit_off[fr] = fr * nq;
        if (fr == n) continue;
        const int32_t ti = (int32_t)(fr / f.n_rows);
        int32_t mode = row_mode[fr % f.n_rows];
        if (mode < 0 || mode >= n_modes) {
            raise_flag(flag);
            mode = -1;
        }
        RowInfo ri;
        ri.rec = nullptr;
        ri.beg = ri.end = 0;
        ri.hbase = 0;
        ri.mode = mode;
        ri.type = f.types[ti];
        rows[fr] = ri;
    }
}

// n-th (0-based) set bit of w; w has more than n set bits.
__device__ inline int select_bit(uint64_t w, int n) {
    int pos = 0;
#pragma unroll
    for (int half = 32; half >= 1; half >>= 1) {
        const uint64_t lo = w & ((1ull << half) - 1);
        const int c = __popcll(lo);
        if (n >= c) {
            n -= c;
            w >>= half;
            pos += half;
        }
    }
    return pos;
}

// MIXED: the kept records are evaluated by the mixed-precision batch (split
// bf16 MFMA build, FP32 contraction, FP64 weights) instead of the FP64 one.
template <int MAXT, bool ADAPT, bool MIXED>
__global__ __launch_bounds__(kBlock, MIXED ? 2 : 3) void k_fused4(const double* __restrict__ omega, const double2* __restrict__ evec,
                                                     const double* __restrict__ occ, const double2* __restrict__ roots,
                                                     const double2* __restrict__ phit,
                                                     const int32_t* __restrict__ tmeta,
                                                     const int32_t* __restrict__ groups,
                                                     const RowInfo* __restrict__ rows, double* __restrict__ partial,
                                                     int64_t* __restrict__ unit_kept, int64_t* __restrict__ unit_tup,
                                                     int* __restrict__ flag, RatesArgs a, FusedArgs f, const float2* __restrict__ evec32,
                                                     const uint4* __restrict__ fsp, int32_t n_kblk) {
    constexpr int NB = kFusedNb;
    // dynamic LDS: the root table (FP64, or its bf16 splits: 16 bytes an entry
    // either way), then the term table
    extern __shared__ double2 sroots[];
    __shared__ std::conditional_t<MIXED, float2, double2> sA[kWavesPerBlock][MIXED ? kTB : kFusedTB][27];
    __shared__ int32_t sQ[kWavesPerBlock][MIXED ? kTB : kFusedTB][2];
    const int32_t* tm;
    if constexpr (MIXED) {
        tbm_roots(reinterpret_cast<uint4*>(sroots), roots, a.geo.L);
        tm = tb_stage_terms(sroots + a.geo.L, tmeta, a.n_terms);
    } else {
        tm = tb_stage(sroots, roots, a.geo.L, tmeta, a.n_terms);
    }
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcd;
    const int64_t wstride = (int64_t)(gridDim.x / kXcd) * kWavesPerBlock;
    const ModeGeom geo = a.geo;
    const int32_t N0 = geo.N0, N1 = geo.N1, N2 = geo.N2;
    const int32_t nq = N0 * N1 * N2;
    // Each XCD takes one slice of the q' range of every fused row.  The kept
    // processes per unit differ by orders of magnitude between the types (and
    // between rows), so a contiguous range of units per XCD would leave most
    // XCDs idle while the few holding the +- rows finish; slices of q' spread
    // every row evenly, and consecutive units of an XCD still share a row's
    // force-constant table in its L2.  Unit u = fr * nq + q' keeps its slot in
    // the partials, so the per-row sums keep their order.
    const int32_t q_sl = (nq + kXcd - 1) / kXcd;
    const int32_t q_beg = xcd * q_sl < nq ? xcd * q_sl : nq;
    const int32_t q_cnt = (q_beg + q_sl < nq ? q_beg + q_sl : nq) - q_beg;
    const int64_t w_end = (f.n_units / nq) * q_cnt;
    double dl[MAXT];
#pragma unroll
    for (int it = 0; it < MAXT; ++it) dl[it] = 0.0;

    for (int64_t w = (int64_t)(blockIdx.x / kXcd) * kWavesPerBlock + wave; w < w_end; w += wstride) {
        const int64_t fr = w / q_cnt;
        const int32_t iq1 = q_beg + (int32_t)(w % q_cnt);
        const int64_t u = fr * nq + iq1;
        const RowInfo ri = rows[fr];
        const int32_t g0 = __builtin_amdgcn_readfirstlane(ri.mode);
        const int type = __builtin_amdgcn_readfirstlane(ri.type);
        double accg[MAXT], accw[MAXT];
#pragma unroll
        for (int it = 0; it < MAXT; ++it) accg[it] = accw[it] = 0.0;
        int64_t kept = 0;
        int64_t ntup = 0;  // (lambda, q', q'') tuples with a kept record
        const double w0 = g0 >= 0 ? omega[g0] : 0.0;
        if (g0 >= 0 && w0 >= f.floor_) {
            int s1, s2, s3;
            type_signs(type, s1, s2, s3);
            const bool tri12 = s1 == s2, tri23 = s2 == s3;
            const int32_t iq0 = g0 / NB;
            const int32_t q00 = iq0 / (N1 * N2), q01 = (iq0 / N2) % N1, q02 = iq0 % N2;
            const int32_t q10 = iq1 / (N1 * N2), q11 = (iq1 / N2) % N1, q12 = iq1 % N2;
            const double2* __restrict__ phit_row = phit + fr * a.n_terms * 27;
            double w1[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) w1[j] = omega[iq1 * NB + j];
            double pm1[3] = {0.0, 0.0, 0.0};
            if (ADAPT) fused_proj_max(f.vel, iq1, f, geo, pm1);

            // kept records wait in buf (position k * 64 + lane in buf[k], pend of
            // them) until 128 have gathered, across chunks of q''; one pass past
            // the last chunk (no candidates) evaluates the remainder
            uint64_t buf[kBR];
#pragma unroll
            for (int k = 0; k < kBR; ++k) buf[k] = 0;
            int pend = 0;
            for (int32_t start = tri12 ? iq1 : 0;; start += kWave) {
                const bool last = start >= nq;
                // ---- candidate masks: lane = q''
                const int32_t iq2 = start + lane;
                const bool qv = iq2 < nq;
                uint64_t m[4] = {0, 0, 0, 0};
                if (qv) {
                    const int32_t q20 = iq2 / (N1 * N2), q21 = (iq2 / N2) % N1, q22 = iq2 % N2;
                    // s3 q''' = -(q + s1 q' + s2 q'')
                    const int32_t iq3 = (wrapn(s3 * -(q00 + s1 * q10 + s2 * q20), N0) * N1 +
                                         wrapn(s3 * -(q01 + s1 * q11 + s2 * q21), N1)) * N2 +
                                        wrapn(s3 * -(q02 + s1 * q12 + s2 * q22), N2);
                    double w2[NB], w3[NB];
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        w2[j] = omega[iq2 * NB + j];
                        w3[j] = omega[iq3 * NB + j];
                    }
                    // adaptive width: a bound for this triple of q-points, so the
                    // exact width is evaluated only where it can matter
                    double cut_q = f.cut;
                    uint64_t xm[4] = {0, 0, 0, 0};  // candidates that need the exact width
                    if (ADAPT) {
                        double pm2[3], pm3[3];
                        fused_proj_max(f.vel, iq2, f, geo, pm2);
                        fused_proj_max(f.vel, iq3, f, geo, pm3);
                        cut_q = fused_cut_bound(pm1, pm2, pm3, f);
                    }
#pragma unroll
                    for (int j1 = 0; j1 < NB; ++j1) {
                        const int32_t g1 = iq1 * NB + j1;
                        const bool ok1 = w1[j1] >= f.floor_;
                        const double d1 = s1 > 0 ? w0 + w1[j1] : w0 - w1[j1];
#pragma unroll
                        for (int j2 = 0; j2 < NB; ++j2) {
                            const int32_t g2 = iq2 * NB + j2;
                            const bool ok2 = ok1 && !(tri12 && g2 < g1) && w2[j2] >= f.floor_;
                            const double d2 = s2 > 0 ? d1 + w2[j2] : d1 - w2[j2];
#pragma unroll
                            for (int j3 = 0; j3 < NB; ++j3) {
                                const int32_t g3 = iq3 * NB + j3;
                                const double delta = s3 > 0 ? d2 + w3[j3] : d2 - w3[j3];
                                bool keep = ok2 && !(tri23 && g3 < g2) && w3[j3] >= f.floor_;
                                bool exact = false;
                                if (keep) {
                                    const double ad = fabs(delta);
                                    // sigma_p >= sigma, so the fixed cut keeps without the width
                                    keep = ad <= f.cut;
                                    if (ADAPT) exact = !keep && ad <= cut_q;
                                }
                                const int c = (j1 * NB + j2) * NB + j3;
                                if (keep) m[c >> 6] |= 1ull << (c & 63);
                                if (ADAPT && exact) xm[c >> 6] |= 1ull << (c & 63);
                            }
                        }
                    }
                    // the candidates between the two cuts: each lane walks its own
                    // set bits, two at a time so that the table reads of both are in
                    // flight together (the walk waits on memory, not arithmetic), and
                    // the wave runs as many steps as its busiest lane needs rather than
                    // one per candidate position any lane needs.  The mismatch is
                    // formed again with the same operations in the same order, so the
                    // decision is the one the host makes.
                    if (ADAPT) {
#pragma unroll
                        for (int wd = 0; wd < 4; ++wd) {
                            uint64_t xb = xm[wd];
                            const int bit0 = xb ? __builtin_ctzll(xb) : 0;  // a real candidate, for idle slots
                            while (xb) {
                                int bit[2];
                                bool cv[2];
#pragma unroll
                                for (int k = 0; k < 2; ++k) {
                                    cv[k] = xb != 0;
                                    bit[k] = cv[k] ? __builtin_ctzll(xb) : bit0;
                                    xb &= xb - 1;
                                }
                                double ad[2], nrm[2];
                                int32_t ga[2], gb[2], gc[2];
#pragma unroll
                                for (int k = 0; k < 2; ++k) {
                                    const int c = wd * 64 + bit[k];
                                    const int j1 = c / (NB * NB), j2 = (c / NB) % NB, j3 = c % NB;
                                    ga[k] = iq1 * NB + j1;
                                    gb[k] = iq2 * NB + j2;
                                    gc[k] = iq3 * NB + j3;
                                    double o1 = w1[0], o2 = w2[0], o3 = w3[0];
#pragma unroll
                                    for (int j = 1; j < NB; ++j) {
                                        o1 = j1 == j ? w1[j] : o1;
                                        o2 = j2 == j ? w2[j] : o2;
                                        o3 = j3 == j ? w3[j] : o3;
                                    }
                                    const double d1 = s1 > 0 ? w0 + o1 : w0 - o1;
                                    const double d2 = s2 > 0 ? d1 + o2 : d1 - o2;
                                    const double delta = s3 > 0 ? d2 + o3 : d2 - o3;
                                    ad[k] = fabs(delta);
                                    nrm[k] = __builtin_sqrt(proj_sq(a.br.proj, ga[k], gb[k]) +
                                                            proj_sq(a.br.proj, ga[k], gc[k]) +
                                                            proj_sq(a.br.proj, gb[k], gc[k]));
                                }
#pragma unroll
                                for (int k = 0; k < 2; ++k) {
                                    // the width from the per-mode projection table brackets the
                                    // enumerator's; only a candidate inside the bracket needs
                                    // the enumerator's own arithmetic
                                    constexpr double rel = 1e-13;
                                    const double sp_lo = f.factor / 3.0 * (nrm[k] * (1.0 - rel) - f.perr) * (1.0 - rel);
                                    const double sp_hi = f.factor / 3.0 * (nrm[k] * (1.0 + rel) + f.perr) * (1.0 + rel);
                                    const double thr_lo = f.nsigma * fmax(sp_lo, f.sigma) * (1.0 - rel);
                                    const double thr_hi = f.nsigma * fmax(sp_hi, f.sigma) * (1.0 + rel);
                                    bool keep = ad[k] <= thr_lo;
                                    if (cv[k] && !keep && ad[k] <= thr_hi)
                                        keep = fused_adaptive_pass(ad[k], ga[k], gb[k], gc[k], f, geo);
                                    if (cv[k] && keep) m[wd] |= 1ull << bit[k];
                                }
                            }
                        }
                    }
                }
                const int cnt = __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2]) + __popcll(m[3]);
                // inclusive prefix over the wave
                int incl = cnt;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) {
                    const int v = __shfl_up(incl, d, kWave);
                    if (lane >= d) incl += v;
                }
                const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1, kWave));
                const int excl = incl - cnt;
                kept += total;
                ntup += __popcll(__ballot(cnt > 0));
                // ---- batches of 128 kept records, in (q'', j', j'', j''') order
                int used = 0;
                do {
                    const int take = kBU - pend < total - used ? kBU - pend : total - used;
                    if (take > 0) {
#pragma unroll
                        for (int k = 0; k < kBR; ++k) {
                            // every lane decodes (clamped), so the shuffles see the whole wave
                            const int pos = k * kWave + lane;
                            const int p = used + pos - pend;
                            const int pc = p < 0 ? 0 : (p < total ? p : total - 1);
                            int lo = 0, hi = kWave - 1;  // largest lane s with excl[s] <= pc
#pragma unroll
                            for (int it = 0; it < 6; ++it) {
                                const int mid = (lo + hi + 1) >> 1;
                                if (__shfl(excl, mid, kWave) <= pc)
                                    lo = mid;
                                else
                                    hi = mid - 1;
                            }
                            int n = pc - __shfl(excl, lo, kWave);
                            uint64_t w[4];
#pragma unroll
                            for (int x = 0; x < 4; ++x) w[x] = __shfl(m[x], lo, kWave);
                            // word holding the n-th set bit, then the bit within it
                            uint64_t ww = w[0];
                            int word = 0;
#pragma unroll
                            for (int x = 0; x < 3; ++x) {
                                const int c = __popcll(ww);
                                if (word == x && n >= c) {
                                    n -= c;
                                    word = x + 1;
                                    ww = w[x + 1];
                                }
                            }
                            const int c = word * 64 + select_bit(ww, n);
                            const int j1 = c / (NB * NB), j2 = (c / NB) % NB, j3 = c % NB;
                            const uint64_t g1 = (uint64_t)(iq1 * NB + j1);
                            const uint64_t g2 = (uint64_t)((start + lo) * NB + j2);
                            if (pos >= pend && pos < pend + take) buf[k] = g1 | (g2 << 24) | ((uint64_t)j3 << 48);
                        }
                    }
                    pend += take;
                    used += take;
                    if (pend == kBU || (last && pend > 0)) {
                        if constexpr (MIXED)
                            tbm_batch<MAXT, false>(buf, pend, g0, type, fsp + fr * n_kblk * 4 * kWave * 3, omega,
                                                   evec32, occ, tm, groups, flag, a,
                                                   reinterpret_cast<const uint4*>(sroots), sA[wave], sQ[wave], accg,
                                                   accw, dl, 0.0, nullptr);
                        else
                            tb_batch<MAXT, false, kBR, kFusedTB>(buf, pend, g0, type, phit_row, omega, evec, occ, tm, groups, flag, a,
                                                  sroots, sA[wave], sQ[wave], accg, accw, dl, 0.0, nullptr);
                        pend = 0;
                    }
                } while (used < total);
                if (last) break;
            }
        }
        double* out = partial + u * (2 * a.n_T);
#pragma unroll
        for (int it = 0; it < MAXT; ++it) {
            if (it < a.n_T) {
                const double sg = wave_sum(accg[it]);
                const double sw = wave_sum(accw[it]);
                if (lane == 0) {
                    out[it] = sg;
                    out[a.n_T + it] = sw;
                }
            }
        }
        if (lane == 0) {
            unit_kept[u] = kept;
            unit_tup[u] = ntup;
        }
    }
}

// out[0] = sum of v[0..n), one block, fixed order.
__global__ void k_sum_i64(const int64_t* __restrict__ v, int64_t n, int64_t* __restrict__ out) {
    __shared__ int64_t red[kBlock];
    int64_t s = 0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace fpk
