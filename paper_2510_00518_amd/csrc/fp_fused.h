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
    const double* proj;      // the per-mode table (proj_0, proj_1, proj_2, omega)
    const double* proj_max;  // per q-point: the largest |proj_d| over its branches
    double recip[9];
    double factor, sigma, nsigma, cut_max;
    double wmin, wmax;  // smallest active and largest frequency of the mesh (unit bound)
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

// The enumerator's own width test, for the candidates inside the bracket of
// the table width (rare).  Inlined: as a call it cost the kernel a call frame
// and register saves around the walk (8.60 s against 7.55 s for the 16^3 cell).
__device__ inline bool fused_adaptive_pass(double ad, int32_t g1, int32_t g2, int32_t g3, const FusedArgs& f,
                                           const ModeGeom& geo) {
#pragma clang fp contract(off)
    double s2 = fused_pair_sq(0.0, f.vel, g1, g2, f, geo);
    s2 = fused_pair_sq(s2, f.vel, g1, g3, f, geo);
    s2 = fused_pair_sq(s2, f.vel, g2, g3, f, geo);
    const double sp = f.factor * __builtin_sqrt(s2 / 9.0);
    return ad <= f.nsigma * (sp > f.sigma ? sp : f.sigma);
}

// ---------------------------------------------------------------------------
// FP64 form with the first partner folded per unit.  Within a unit (lambda, q')
// the partner lambda' = (q', j') ranges over the branches of q' only, so its
// eigenvector and the phase exp(2 pi i Q1.A_k / L) of every phase key k are
// fixed.  Folding both into the force constants once per unit gives, per pair
// group p (the atoms c, d of slots 2 and 3) and pkey (a distinct B in p),
//   H_p[pk][j' gamma delta] = sum_{k in pk} exp(2 pi i Q1.A_k/L)
//                             sum_beta phit_k[beta gamma delta] eps1(j', b_k)_beta,
// so the keys of the two slot-1 atoms share one table.  Per tuple tau (q'', and
// with it the last partner's q, fixed) the build on FP64 MFMA is
//   A_p[j' gamma delta](tau) = sum_{pk in p} exp(2 pi i Q2(tau).B_pk / L) H_p[pk][j' gamma delta]
// (M = 54 components in four tiles, N = 16 tuples, K = the pkeys, four at a
// time), and each process contracts
//   V = sum_p sum_{gamma delta} A_p[j' gamma delta](tau) eps2(c_p)_gamma eps3(d_p)_delta,
// 12 complex MACs per pair group against 39 per partner-atom group without the fold.
constexpr int kXM = 54;   // components j' gamma delta of one pair group
constexpr int kXMT = 4;   // M-tiles of 16
constexpr int kXTB = 16;  // tuples per batch tile (the MFMA N)

// H of this unit for every pkey, written to the block's LDS table sF[pk][54]
// (component j' * 9 + gamma delta) by all threads of the block together, in
// FP64 and stored as TF (double2, or float2 for the mixed form).  c1 = +1 or -1
// conjugates the eigenvectors of an emitted lambda'.
template <class TF>
__device__ inline void tbx_fold(TF* sF, int32_t n_pkeys, const double2* __restrict__ phit_row,
                                const double2* __restrict__ evec, int32_t iq1, double c1, int32_t Q10, int32_t Q11,
                                int32_t Q12, const int32_t* __restrict__ tm, const int32_t* __restrict__ ptab,
                                const int32_t* __restrict__ plist, const double2* sroots, const ModeGeom& geo) {
    const int nb = geo.nb;
    for (int i = threadIdx.x; i < n_pkeys * kXM; i += kBlock) {
        const int32_t pk = i / kXM;
        const int mc = i % kXM;
        const int jp = mc / 9, gd = mc % 9;
        const int32_t e0 = ptab[pk * 8], e1 = e0 + ptab[pk * 8 + 1];
        double2 F = make_double2(0.0, 0.0);
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t k = plist[2 * e], ab = plist[2 * e + 1];
            const int32_t* t = tm + k * 8;
            const uint32_t kq = (uint32_t)(Q10 * t[1] + Q11 * t[2] + Q12 * t[3]);
            const double2* x = evec + ((int64_t)iq1 * nb + jp) * nb + 3 * ab;
            const double2* h = phit_row + (int64_t)k * 27 + gd;
            double2 hx = make_double2(0.0, 0.0);
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) hx = cfma(hx, h[bb * 9], ld_eps(x + bb, c1));
            F = cfma(F, sroots[mod_l(kq, geo.L, geo.magic)], hx);
        }
        if constexpr (sizeof(TF) == sizeof(float2))
            sF[i] = make_float2((float)F.x, (float)F.y);
        else
            sF[i] = F;
    }
}

// One record of the form-2 batch: the three partner modes and the branch of the
// first partner (g1 = g0 for a slot without a record).
struct XProc {
    int32_t g1, g2, gl, jp;
};

// Form-2 records, written by the fused filter: j1 | j2 << 3 | j3 << 6 |
// iq2 << 9 | iq3 << 33, with q' the unit's (iq1) and the last partner's q-point
// iq3 already closed by momentum, so no index division is left here.
__device__ inline XProc tbx_decode(bool have, uint64_t rec, int32_t g0, int32_t iq1) {
    XProc p;
    p.g1 = p.g2 = p.gl = g0;
    p.jp = 0;
    if (!have) return p;
    const int j1 = (int)(rec & 7u), j2 = (int)((rec >> 3) & 7u), j3 = (int)((rec >> 6) & 7u);
    const int32_t iq2 = (int32_t)((rec >> 9) & 0xFFFFFFu), iq3 = (int32_t)((rec >> 33) & 0xFFFFFFu);
    p.g1 = iq1 * kFusedNb + j1;
    p.g2 = iq2 * kFusedNb + j2;
    p.gl = iq3 * kFusedNb + j3;
    p.jp = j1;
    return p;
}

// The weight factor w G(Delta) / prod(omega) of a decoded record (w the
// triangle weight, G the Gaussian of the call's or the adaptive width), formed
// after the contraction so that it holds no registers there; the mismatch, the
// product of frequencies and the width follow setup_proc's operation order.
__device__ inline double tbx_weight(const XProc& p, int type, int s1, int s2, int s3, double w0,
                                    const double* __restrict__ omega, const Broad& br) {
    Proj4 P1, P2, Pl;
    double w1, w2, wl;
    if (br.proj) {  // the adaptive width's table rows carry the frequencies too
        P1 = ld_proj4(br.proj, p.g1);
        P2 = ld_proj4(br.proj, p.g2);
        Pl = ld_proj4(br.proj, p.gl);
        w1 = P1.b.y;
        w2 = P2.b.y;
        wl = Pl.b.y;
    } else {
        w1 = omega[p.g1];
        w2 = omega[p.g2];
        wl = omega[p.gl];
    }
    double delta = s1 > 0 ? w0 + w1 : w0 - w1;
    delta = s2 > 0 ? delta + w2 : delta - w2;
    delta = s3 > 0 ? delta + wl : delta - wl;
    double wprod = w0 * w1 * w2;
    wprod *= wl;
    double wt = 1.0;
    if (type == 2) {
        if (p.g1 == p.g2) wt = 0.5;
    } else if (type == 3) {
        if (p.g2 == p.gl) wt = 0.5;
    } else {
        const int eq = (p.g1 == p.g2) + (p.g2 == p.gl) + (p.g1 == p.gl);
        wt = eq == 3 ? (1.0 / 6.0) : (eq >= 1 ? 0.5 : 1.0);
    }
    double inv_sigma2 = br.inv_sigma2, gnorm = br.gnorm;
    if (br.proj) {
        const double s2q = proj_sq4(P1, P2) + proj_sq4(P1, Pl) + proj_sq4(P2, Pl);
        const double sig = fmax(br.factor * sqrt(s2q * (1.0 / 9.0)), br.floor_);
        inv_sigma2 = 1.0 / (sig * sig);
        gnorm = 0.56418958354775628695 / sig;  // 1/(sigma sqrt(pi))
    }
    return wt * exp(-(delta * delta) * inv_sigma2) * gnorm / wprod;
}

// One batch of up to 128 records of one unit (record k * 64 + lane in rec[k];
// `count` valid), all with the unit's q': decode, find the tuples (a change of
// q'' between consecutive records), build A_p per pair group and 16-tuple tile
// on FP64 MFMA from the block's folded table sF, contract per process on the VALU,
// weight in FP64.  ptab is the pkey table (B at [4..6]); A and Qs are this
// wave's LDS staging.
template <int MAXT, bool F32>
__device__ inline void tbx_batch(const uint64_t (&rec)[kBR], const int32_t (&qpk)[kBR], int count, int32_t g0,
                                 int type, int32_t iq1, const std::conditional_t<F32, float2, double2>* sF,
                                 const double* __restrict__ omega, const double2* __restrict__ evec,
                                 const float2* __restrict__ evec32,
                                 const double* __restrict__ occt, const int32_t* __restrict__ ptab,
                                 const int32_t* __restrict__ pgroups, int n_pgroups, const RatesArgs& a,
                                 const double2* sroots, std::conditional_t<F32, float2, double2> (*A)[kXM],
                                 int32_t* Qs, double (&accg)[MAXT], double (&accw)[MAXT]) {
    constexpr int MT = (MAXT + 1) & ~1;  // occupations per mode in occt (temperature-fastest)
    const int lane = threadIdx.x & (kWave - 1);
    const int li = lane & 15, lk = lane >> 4;
    const ModeGeom& geo = a.geo;
    const int nb = geo.nb;
    int s1, s2, s3;
    type_signs(type, s1, s2, s3);
    const double c2 = s2 > 0 ? 1.0 : -1.0;
    const double c3 = s3 > 0 ? 1.0 : -1.0;
    const double w0 = omega[g0];

    // ---- records, tuple boundaries (q'' changes) and slots
    XProc pr[kBR];
    bool have[kBR], first[kBR];
    int slot[kBR];
    int32_t prev_last = -1;
    int base = 0;
#pragma unroll
    for (int k = 0; k < kBR; ++k) {
        const int idx = k * kWave + lane;
        have[k] = idx < count;
        pr[k] = tbx_decode(have[k], rec[k], g0, iq1);
        const int32_t key = have[k] ? (int32_t)((rec[k] >> 9) & 0xFFFFFFu) : -2;
        int32_t up = __shfl(key, (lane + kWave - 1) & (kWave - 1), kWave);
        if (lane == 0) up = prev_last;
        first[k] = have[k] && key != up;
        const uint64_t mask = __ballot(first[k]);
        const uint64_t le = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
        slot[k] = base + __popcll(mask & le) - 1;
        base += __popcll(mask);
        prev_last = __shfl(key, kWave - 1, kWave);
    }
    const int n_tup = __builtin_amdgcn_readfirstlane(base);

    double2 V[kBR];
#pragma unroll
    for (int k = 0; k < kBR; ++k) V[k] = make_double2(0.0, 0.0);
    for (int gi = 0; gi < n_pgroups; ++gi) {
        const int32_t* G = pgroups + gi * 8;
        const int32_t ac = G[0], ad = G[1], p0 = G[2], p1 = G[3];
        const int n_ks = (p1 - p0 + 3) >> 2;  // <= kMaxKs: groups hold at most 16 pkeys
        for (int tb = 0; tb < n_tup; tb += kXTB) {
            const int nbt = n_tup - tb < kXTB ? n_tup - tb : kXTB;
            if (gi == 0 || n_tup > kXTB) {  // one tile: the staged q'' of the first group serve all
#pragma unroll
                for (int k = 0; k < kBR; ++k) {
                    const int s = slot[k] - tb;
                    if (first[k] && s >= 0 && s < kXTB) Qs[s] = qpk[k];
                }
                lds_fence();
            }
            // A_p for this tile: two passes of two M-tiles (Karatsuba, three real
            // MFMAs per complex product: k1 = (Fr + Fi) pr, k2 = Fr (pi - pr),
            // k3 = Fi (pr + pi); Re = k1 - k3, Im = k1 + k2)
            // FP64: the partner slices of slots 2 and 3 are gathered before the
            // A_p build, so their L2 latency overlaps the matrix work (a record
            // outside this tile, or a padding slot, reads a valid mode and is unused)
            double2 yv[kBR][3], zv[kBR][3];
            if constexpr (!F32) {
#pragma unroll
                for (int k = 0; k < kBR; ++k) {
                    const double2* e2 = evec + (int64_t)pr[k].g2 * nb + 3 * ac;
                    const double2* e3 = evec + (int64_t)pr[k].gl * nb + 3 * ad;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        yv[k][q] = ld_eps(e2 + q, c2);
                        zv[k][q] = ld_eps(e3 + q, c3);
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
            const bool tval = li < nbt;
            const int32_t qa = Qs[tval ? li : 0];
            const int32_t qb0 = qa & 1023, qb1 = (qa >> 10) & 1023, qb2 = (qa >> 20) & 1023;
if constexpr (F32) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                f4v k1[2], k2[2], k3[2];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) k1[mt] = k2[mt] = k3[mt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < kMaxKs; ++ks) {
                    if (ks >= n_ks) break;
                    const int32_t pk = p0 + 4 * ks + lk;
                    float2 ph = make_float2(0.0f, 0.0f);
                    if (pk < p1 && tval) {
                        const int32_t* b = ptab + pk * 8;
                        const uint32_t kq = (uint32_t)(qb0 * b[4] + qb1 * b[5] + qb2 * b[6]);
                        const double2 r = sroots[mod_l(kq, geo.L, geo.magic)];
                        ph = make_float2((float)r.x, (float)r.y);
                    }
                    const float pd = ph.y - ph.x, ps = ph.x + ph.y;
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        const int mc = (2 * half + mt) * 16 + li;
                        const float2 F = pk < p1 && mc < kXM ? sF[pk * kXM + mc] : make_float2(0.0f, 0.0f);
                        k1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(F.x + F.y, ph.x, k1[mt], 0, 0, 0);
                        k2[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(F.x, pd, k2[mt], 0, 0, 0);
                        k3[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(F.y, ps, k3[mt], 0, 0, 0);
                    }
                }
                // FP32 result layout: D[i = 4 lk + r][j = li]
                if (tval) {
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int mc = (2 * half + mt) * 16 + 4 * lk + r;
                            if (mc < kXM) A[li][mc] = make_float2(k1[mt][r] - k3[mt][r], k1[mt][r] + k2[mt][r]);
                        }
                }
            }
            } else {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                d4 k1[2], k2[2], k3[2];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) k1[mt] = k2[mt] = k3[mt] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < kMaxKs; ++ks) {
                    if (ks >= n_ks) break;
                    const int32_t pk = p0 + 4 * ks + lk;
                    double2 ph = make_double2(0.0, 0.0);
                    if (pk < p1 && tval) {
                        const int32_t* b = ptab + pk * 8;
                        const uint32_t kq = (uint32_t)(qb0 * b[4] + qb1 * b[5] + qb2 * b[6]);
                        ph = sroots[mod_l(kq, geo.L, geo.magic)];
                    }
                    const double pd = ph.y - ph.x, ps = ph.x + ph.y;
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        const int mc = (2 * half + mt) * 16 + li;
                        const double2 F = pk < p1 && mc < kXM ? sF[pk * kXM + mc] : make_double2(0.0, 0.0);
                        k1[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.x + F.y, ph.x, k1[mt], 0, 0, 0);
                        k2[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.x, pd, k2[mt], 0, 0, 0);
                        k3[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.y, ps, k3[mt], 0, 0, 0);
                    }
                }
                // D[i = 4r + lk][j = li]: component (2 half + mt) 16 + 4r + lk of tuple li
                if (tval) {
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int mc = (2 * half + mt) * 16 + 4 * r + lk;
                            if (mc < kXM) A[li][mc] = make_double2(k1[mt][r] - k3[mt][r], k1[mt][r] + k2[mt][r]);
                        }
                }
            }
            }
            lds_fence();
            __builtin_amdgcn_s_setprio(3);
            // per process: 9 + 3 complex MACs with the partners of slots 2 and 3
#pragma unroll
            for (int k = 0; k < kBR; ++k) {
                const int s = slot[k] - tb;
                if (have[k] && s >= 0 && s < nbt) {
                    if constexpr (F32) {
                        const float2* e2 = evec32 + (int64_t)pr[k].g2 * nb + 3 * ac;
                        const float2* e3 = evec32 + (int64_t)pr[k].gl * nb + 3 * ad;
                        float2 y[3], z[3];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            y[q] = ld_eps32(e2 + q, (float)c2);
                            z[q] = ld_eps32(e3 + q, (float)c3);
                        }
                        const float2* Ar = A[s] + pr[k].jp * 9;
                        float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            float2 vc = make_float2(0.0f, 0.0f);
#pragma unroll
                            for (int d = 0; d < 3; ++d) vc = cfmaf(vc, Ar[c * 3 + d], z[d]);
                            acc = cfmaf(acc, vc, y[c]);
                        }
                        V[k].x += (double)acc.x;
                        V[k].y += (double)acc.y;
                    } else {
                        const double2(&y)[3] = yv[k];
                        const double2(&z)[3] = zv[k];
                        const double2* Ar = A[s] + pr[k].jp * 9;
                        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double2 vc = make_double2(0.0, 0.0);
#pragma unroll
                            for (int d = 0; d < 3; ++d) vc = cfma(vc, Ar[c * 3 + d], z[d]);
                            acc = cfma(acc, vc, y[c]);
                        }
                        V[k].x += acc.x;
                        V[k].y += acc.y;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            lds_fence();
        }
    }

    // ---- weights and occupations (FP64); the three partners' occupations at every
    // temperature come in 16-byte loads from the temperature-fastest table
#pragma unroll
    for (int k = 0; k < kBR; ++k) {
        const double V2 = V[k].x * V[k].x + V[k].y * V[k].y;
        const double base = have[k] ? tbx_weight(pr[k], type, s1, s2, s3, w0, omega, a.br) : 0.0;
        double n1[MT], n2[MT], nl[MT];
#pragma unroll
        for (int it = 0; it < MT; it += 2) {
            const double2 x1 = *reinterpret_cast<const double2*>(occt + (int64_t)pr[k].g1 * MT + it);
            const double2 x2 = *reinterpret_cast<const double2*>(occt + (int64_t)pr[k].g2 * MT + it);
            const double2 xl = *reinterpret_cast<const double2*>(occt + (int64_t)pr[k].gl * MT + it);
            n1[it] = x1.x; n1[it + 1] = x1.y;
            n2[it] = x2.x; n2[it + 1] = x2.y;
            nl[it] = xl.x; nl[it + 1] = xl.y;
        }
#pragma unroll
        for (int it = 0; it < MAXT; ++it) {
            if (it < a.n_T) {
                double oc;
                if (type == 2)
                    oc = n1[it] * n2[it] * (1.0 + nl[it]) - (1.0 + n1[it]) * (1.0 + n2[it]) * nl[it];
                else if (type == 3)
                    oc = n1[it] * (1.0 + n2[it]) * (1.0 + nl[it]) - (1.0 + n1[it]) * n2[it] * nl[it];
                else
                    oc = (1.0 + n1[it]) * (1.0 + n2[it]) * (1.0 + nl[it]) - n1[it] * n2[it] * nl[it];
                const double xw = base * oc;
                accw[it] += xw;
                accg[it] += xw * V2;
            }
        }
    }
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

// Tables of the FP64 forms of the fused kernel (built by fp_load_ifc): the
// B-key form (FORM 0: keys folded over A per unit, tb_batch) and the x-folded
// form (FORM 2: keys and the first partner folded per unit, tbx_batch); fold
// is one table per wave, rewritten per unit, of n_fold_ks K-steps.
struct FusedTabs {
    const int32_t* btab;
    const int32_t* fgroups;
    const int32_t* ptab;
    const int32_t* plist;
    const int32_t* pgroups;
    double2* fold;
    const double* occt;  // form 2: occupations [mode][temperature], rows padded to an even count
    int32_t n_bkeys, n_pkeys, n_pgroups, n_fold_ks;
};

// occt[g * mt + it] = occ[it * n_modes + g], zero in the padding columns it >= n_T
__global__ void k_occ_t(const double* __restrict__ occ, int64_t n_modes, int32_t n_T, int32_t mt,
                        double* __restrict__ occt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_modes * mt;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = i / mt;
        const int it = (int)(i % mt);
        occt[i] = it < n_T ? occ[(int64_t)it * n_modes + g] : 0.0;
    }
}

// FORM 0: FP64, B-keys (tb_batch, 24-tuple batches, three blocks per CU);
// FORM 1: mixed precision (tbm_batch: split bf16 MFMA build, FP32 contraction,
// FP64 weights); FORM 2: FP64 with the first partner folded (tbx_batch,
// batches of at most 16 tuples, two blocks per CU); FORM 3: form 2 in mixed
// precision (folded table, staging and contraction in FP32, the build on FP32
// matrix cores, the filter and weights in FP64).
template <int MAXT, bool ADAPT, int FORM>
__global__ __launch_bounds__(kBlock, FORM == 0 || FORM == 3 ? 3 : 2) void k_fused4(const double* __restrict__ omega, const double2* __restrict__ evec,
                                                     const double* __restrict__ occ, const double2* __restrict__ roots,
                                                     const double2* __restrict__ phit,
                                                     const int32_t* __restrict__ tmeta,
                                                     const int32_t* __restrict__ groups,
                                                     const RowInfo* __restrict__ rows, double* __restrict__ partial,
                                                     int64_t* __restrict__ unit_kept, int64_t* __restrict__ unit_tup,
                                                     int* __restrict__ flag, RatesArgs a, FusedArgs f, const float2* __restrict__ evec32,
                                                     const uint4* __restrict__ fsp, int32_t n_kblk, FusedTabs ft) {
    constexpr int NB = kFusedNb;
    constexpr bool MIXED = FORM == 1;
    constexpr bool XF = FORM >= 2;   // first partner folded per unit (FP64: 2, mixed: 3)
    constexpr bool X32 = FORM == 3;  // FP32 folded table, staging and contraction
    using XT = std::conditional_t<X32, float2, double2>;
    constexpr int STB = FORM == 1 ? kTB : (FORM == 0 ? kFusedTB : kXTB);  // tuples staged per wave
    constexpr int SNC = XF ? kXM : 27;                                    // components staged per tuple
    // dynamic LDS: the root table (FP64, or its bf16 splits: 16 bytes an entry
    // either way), then the key table, then (FP64) the B-key or pkey table
    extern __shared__ double2 sroots[];
    __shared__ std::conditional_t<MIXED || X32, float2, double2> sA[kWavesPerBlock][STB][SNC];
    __shared__ int32_t sQ[kWavesPerBlock][STB][2];
    // FORM 2: the unit's folded table, shared by the block's four waves (after
    // the staged tables, 16-byte aligned), and the per-wave unit sums
    __shared__ double sRed[XF ? kWavesPerBlock : 1][2 * MAXT];
    __shared__ int64_t sCnt[XF ? kWavesPerBlock : 1][2];
    const int32_t* tm;
    const int32_t* bt = XF ? ft.ptab : ft.btab;
    XT* sF = nullptr;
    if constexpr (MIXED) {
        tbm_roots(reinterpret_cast<uint4*>(sroots), roots, a.geo.L);
        tm = tb_stage_terms(sroots + a.geo.L, tmeta, a.n_keys);
    } else {
        tm = tb_stage(sroots, roots, a.geo.L, tmeta, a.n_keys);
        const int32_t n_tab = XF ? ft.n_pkeys : ft.n_bkeys;
        const bool staged = a.n_keys <= kStageTerms && n_tab <= kStageTerms;
        if (staged) bt = tb_stage_terms(reinterpret_cast<int32_t*>(sroots + a.geo.L) + a.n_keys * 8, bt, n_tab);
        if (XF)
            sF = reinterpret_cast<XT*>(sroots + a.geo.L + ((staged ? (a.n_keys + n_tab) * 8 : 0) + 3) / 4);
    }
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcd;
    const int64_t wstride = (int64_t)(gridDim.x / kXcd) * kWavesPerBlock;
    const ModeGeom geo = a.geo;
    // this wave's folded force-constant table (FP64 forms), rewritten per unit
    constexpr int FMT = XF ? kXMT : 2;  // M-tiles per K-step of the folded table
    double2* __restrict__ fw = ft.fold + ((int64_t)blockIdx.x * kWavesPerBlock + wave) * ft.n_fold_ks * FMT * kWave;
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

    // FORM 2: a unit per block (the four waves split its q'' range); else a unit per wave
    const int64_t w_first = XF ? (int64_t)(blockIdx.x / kXcd) : (int64_t)(blockIdx.x / kXcd) * kWavesPerBlock + wave;
    const int64_t w_step = XF ? (int64_t)(gridDim.x / kXcd) : wstride;
    for (int64_t w = w_first; w < w_end; w += w_step) {
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
            const double2* __restrict__ phit_row = phit + fr * a.n_keys * 27;
            double w1[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) w1[j] = omega[iq1 * NB + j];
            double w1max = w1[0], w1min = w1[0];
#pragma unroll
            for (int j = 1; j < NB; ++j) {
                w1max = fmax(w1max, w1[j]);
                w1min = fmin(w1min, w1[j]);
            }
            // Unit bound: every mismatch of the unit lies in [lo, hi] (the first
            // partner from the branches of q', the other two from the mesh's extreme
            // frequencies, summed in the filter's order; rounding is monotone).  A
            // unit whose interval misses the widest cut keeps nothing, so it skips
            // the fold and the q'' loop (most ++ and many -- units).
            const double cut_u = (ADAPT ? f.cut_max : f.cut) + 1e-9 * (w0 + w1max + 2.0 * f.wmax);
            double lo = s1 > 0 ? w0 + w1min : w0 - w1max;
            lo = s2 > 0 ? lo + f.wmin : lo - f.wmax;
            lo = s3 > 0 ? lo + f.wmin : lo - f.wmax;
            double hi = s1 > 0 ? w0 + w1max : w0 - w1min;
            hi = s2 > 0 ? hi + f.wmax : hi - f.wmin;
            hi = s3 > 0 ? hi + f.wmax : hi - f.wmin;
            const bool live = lo <= cut_u && hi >= -cut_u;
            if (live) {
            double pm1[3] = {0.0, 0.0, 0.0};
            if (ADAPT)
                for (int d = 0; d < 3; ++d) pm1[d] = f.proj_max[(int64_t)iq1 * 4 + d];
            // The folded table of the FP64 forms is built at the unit's first
            // batch: most units of the ++ and -- types keep no process at all.
            bool folded = false;
            auto fold_unit = [&]() {
                const int32_t Q10 = s1 > 0 ? q10 : wrapn(-q10, N0);
                const int32_t Q11 = s1 > 0 ? q11 : wrapn(-q11, N1);
                const int32_t Q12 = s1 > 0 ? q12 : wrapn(-q12, N2);
                if constexpr (FORM == 0) {
                    // F[b][c] = sum_{k in b} exp(2 pi i Q1.A_k / L) phit_k[c], in the
                    // MFMA A-operand layout that tb_batch reads (K-step, component
                    // tile, lane); zero for a missing key or component
                    const int li = lane & 15, lk = lane >> 4;
                    for (int gi = 0; gi < a.n_groups; ++gi) {
                        const int32_t* G = ft.fgroups + gi * 8;
                        const int32_t b0 = G[3], b1 = G[4], kb = G[5];
                        const int n_ks = (b1 - b0 + 3) >> 2;
                        for (int ks = 0; ks < n_ks; ++ks) {
                            const int32_t b = b0 + 4 * ks + lk;
                            double2 F0 = make_double2(0.0, 0.0), F1 = make_double2(0.0, 0.0);
                            if (b < b1) {
                                const int32_t k0 = bt[b * 8], k1 = k0 + bt[b * 8 + 7];
                                for (int32_t k = k0; k < k1; ++k) {
                                    const int32_t* e = tm + k * 8;
                                    const uint32_t kk = (uint32_t)(Q10 * e[1] + Q11 * e[2] + Q12 * e[3]);
                                    const double2 uu = sroots[mod_l(kk, geo.L, geo.magic)];
                                    F0 = cfma(F0, uu, phit_row[(int64_t)k * 27 + li]);
                                    if (li < 11) F1 = cfma(F1, uu, phit_row[(int64_t)k * 27 + 16 + li]);
                                }
                            }
                            fw[((int64_t)(kb + ks) * 2 + 0) * kWave + lane] = F0;
                            fw[((int64_t)(kb + ks) * 2 + 1) * kWave + lane] = F1;
                        }
                    }
                }
                folded = true;
            };

            if constexpr (XF) {
                // the block folds the unit's table together (it is read by all
                // four waves); the barrier before keeps the previous unit's
                // readers, the one after every writer
                __syncthreads();
                tbx_fold(sF, ft.n_pkeys, phit_row, evec, iq1, s1 > 0 ? 1.0 : -1.0, s1 > 0 ? q10 : wrapn(-q10, N0),
                         s1 > 0 ? q11 : wrapn(-q11, N1), s1 > 0 ? q12 : wrapn(-q12, N2), tm, bt, ft.plist,
                         sroots, geo);
                __syncthreads();
            }
            // kept records wait in buf (position k * 64 + lane in buf[k], pend of
            // them) until 128 have gathered, across chunks of q''; one pass past
            // the last chunk (no candidates) evaluates the remainder
            uint64_t buf[kBR];
            int32_t qbuf[kBR];  // form 2: each record's packed signed q'' coordinates
#pragma unroll
            for (int k = 0; k < kBR; ++k) {
                buf[k] = 0;
                qbuf[k] = 0;
            }
            int pend = 0;
            int ptup = 0;  // tuples in buf (FORM 2 flushes at kXTB of them)
            // FORM 2: wave w of the block takes the chunks w, w + 4, ... of q''
            const int32_t c_first = (tri12 ? iq1 : 0) + (XF ? wave * kWave : 0);
            const int32_t c_step = XF ? kBlock : kWave;
            for (int32_t start = c_first;; start += c_step) {
                const bool last = start >= nq;
                // ---- candidate masks: lane = q''
                const int32_t iq2 = start + lane;
                const bool qv = iq2 < nq;
                uint64_t m[4] = {0, 0, 0, 0};
                int32_t iq3_l = 0, qpk_l = 0;  // this lane's last q-point and packed signed q'' (form 2)
                if (qv) {
                    int32_t q20, q21, q22;
                    q_coords(iq2, geo, q20, q21, q22);
                    // s3 q''' = -(q + s1 q' + s2 q'')
                    const int32_t iq3 = (wrapn(s3 * -(q00 + s1 * q10 + s2 * q20), N0) * N1 +
                                         wrapn(s3 * -(q01 + s1 * q11 + s2 * q21), N1)) * N2 +
                                        wrapn(s3 * -(q02 + s1 * q12 + s2 * q22), N2);
                    if (XF) {
                        iq3_l = iq3;
                        qpk_l = (s2 > 0 ? q20 : wrapn(-q20, N0)) | ((s2 > 0 ? q21 : wrapn(-q21, N1)) << 10) |
                                ((s2 > 0 ? q22 : wrapn(-q22, N2)) << 20);
                    }
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
                        const double2 a2 = *reinterpret_cast<const double2*>(f.proj_max + (int64_t)iq2 * 4);
                        const double2 a3 = *reinterpret_cast<const double2*>(f.proj_max + (int64_t)iq3 * 4);
                        const double pm2[3] = {a2.x, a2.y, f.proj_max[(int64_t)iq2 * 4 + 2]};
                        const double pm3[3] = {a3.x, a3.y, f.proj_max[(int64_t)iq3 * 4 + 2]};
                        cut_q = fused_cut_bound(pm1, pm2, pm3, f);
                    }
                    // Frequency bounds: every mismatch of this lane with branch j1 lies in
                    // [d1 + lo2 + lo3, d1 + hi2 + hi3] (lo_r, hi_r: the extremes of s_r w_r
                    // over the branches), up to rounding far below `marg`.  A block of
                    // candidates whose interval misses [-cut, cut] keeps nothing, so the
                    // wave skips it when none of its lanes can keep one.
                    double mn2 = w2[0], mx2 = w2[0], mn3 = w3[0], mx3 = w3[0];
#pragma unroll
                    for (int j = 1; j < NB; ++j) {
                        mn2 = fmin(mn2, w2[j]);
                        mx2 = fmax(mx2, w2[j]);
                        mn3 = fmin(mn3, w3[j]);
                        mx3 = fmax(mx3, w3[j]);
                    }
                    const double lo2 = s2 > 0 ? mn2 : -mx2, hi2 = s2 > 0 ? mx2 : -mn2;
                    const double lo3 = s3 > 0 ? mn3 : -mx3, hi3 = s3 > 0 ? mx3 : -mn3;
                    const double marg = 1e-9 * (w0 + w1max + mx2 + mx3);
                    const double cmax = (ADAPT ? cut_q : f.cut) + marg;
                    // per lane, once: the signed frequencies of slots 2 and 3 (a - b is
                    // a + (-b), so the mismatch keeps its bits), their floor tests, and
                    // the triangle order of q'' against q' and of q''' against q''
                    double sw2[NB], sw3[NB];
                    bool ok2f[NB], ok3f[NB];
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        sw2[j] = s2 > 0 ? w2[j] : -w2[j];
                        sw3[j] = s3 > 0 ? w3[j] : -w3[j];
                        ok2f[j] = w2[j] >= f.floor_;
                        ok3f[j] = w3[j] >= f.floor_;
                    }
                    const bool lt21 = iq2 < iq1, eq21 = iq2 == iq1;
                    const double lo23 = lo2 + lo3, hi23 = hi2 + hi3;  // pruning bounds (the margin covers the regrouping)
                    const bool lt32 = iq3 < iq2, eq32 = iq3 == iq2;
#pragma unroll
                    for (int j1 = 0; j1 < NB; ++j1) {
                        const bool ok1 = w1[j1] >= f.floor_;
                        const double d1 = s1 > 0 ? w0 + w1[j1] : w0 - w1[j1];
                        if (!__ballot(ok1 && d1 + lo23 <= cmax && d1 + hi23 >= -cmax)) continue;
#pragma unroll
                        for (int j2 = 0; j2 < NB; ++j2) {
                            // g2 < g1 <=> q'' before q', or the same q-point and j'' < j'
                            const bool below1 = lt21 || (eq21 && j2 < j1);
                            const bool ok2 = ok1 && !(tri12 && below1) && ok2f[j2];
                            const double d2 = d1 + sw2[j2];
                            if (!__ballot(ok2 && d2 + lo3 <= cmax && d2 + hi3 >= -cmax)) continue;
#pragma unroll
                            for (int j3 = 0; j3 < NB; ++j3) {
                                const bool below2 = lt32 || (eq32 && j3 < j2);
                                const double ad = fabs(d2 + sw3[j3]);
                                const bool ok = ok2 && !(tri23 && below2) && ok3f[j3];
                                // sigma_p >= sigma, so the fixed cut keeps without the width
                                const bool keep = ok && ad <= f.cut;
                                const int c = (j1 * NB + j2) * NB + j3;
                                if (keep) m[c >> 6] |= 1ull << (c & 63);
                                if (ADAPT && ok && !keep && ad <= cut_q) xm[c >> 6] |= 1ull << (c & 63);
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
                        uint64_t x0 = xm[0], x1 = xm[1], x2 = xm[2], x3 = xm[3];
                        while (x0 | x1 | x2 | x3) {
                            int cc[2];
                            bool cv[2];
#pragma unroll
                            for (int k = 0; k < 2; ++k) {
                                // lowest pending candidate over the four words (an idle
                                // second slot repeats the first, its result unused)
                                cv[k] = (x0 | x1 | x2 | x3) != 0;
                                const int wd = x0 ? 0 : (x1 ? 1 : (x2 ? 2 : 3));
                                const uint64_t cur = x0 ? x0 : (x1 ? x1 : (x2 ? x2 : x3));
                                cc[k] = cv[k] ? wd * 64 + __builtin_ctzll(cur) : cc[0];
                                const uint64_t nxt = cur & (cur - 1);
                                x0 = wd == 0 ? nxt : x0;
                                x1 = wd == 1 ? nxt : x1;
                                x2 = wd == 2 ? nxt : x2;
                                x3 = wd == 3 ? nxt : x3;
                            }
                            double ad[2], nrm[2];
                            int32_t ga[2], gb[2], gc[2];
#pragma unroll
                            for (int k = 0; k < 2; ++k) {
                                const int c = cc[k];
                                const int j1 = c / (NB * NB), j2 = (c / NB) % NB, j3 = c % NB;
                                ga[k] = iq1 * NB + j1;
                                gb[k] = iq2 * NB + j2;
                                gc[k] = iq3 * NB + j3;
                                const Proj4 P1 = ld_proj4(f.proj, ga[k]), P2 = ld_proj4(f.proj, gb[k]),
                                            P3 = ld_proj4(f.proj, gc[k]);
                                const double d1 = s1 > 0 ? w0 + P1.b.y : w0 - P1.b.y;
                                const double d2 = s2 > 0 ? d1 + P2.b.y : d1 - P2.b.y;
                                const double delta = s3 > 0 ? d2 + P3.b.y : d2 - P3.b.y;
                                ad[k] = fabs(delta);
                                nrm[k] = __builtin_sqrt(proj_sq4(P1, P2) + proj_sq4(P1, P3) + proj_sq4(P2, P3));
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
                                const uint64_t b = cv[k] && keep ? 1ull << (cc[k] & 63) : 0ull;
#pragma unroll
                                for (int x = 0; x < 4; ++x) m[x] |= (cc[k] >> 6) == x ? b : 0ull;
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
                const uint64_t nz = __ballot(cnt > 0);  // lanes (tuples) with kept records
                do {
                    int take = kBU - pend < total - used ? kBU - pend : total - used;
                    if (XF && take > 0) {
                        // at most kXTB - ptup more tuples: every lane the take touches is
                        // one new tuple of the buffer (a take starts at a lane boundary,
                        // or mid-lane right after a flush)
                        const uint64_t from = __ballot(incl > used) & nz;  // lanes at or after record `used`
                        const int room = kXTB - ptup;
                        if (__popcll(from) > room) {
                            const int l1 = select_bit(from, room - 1);  // the room-th such lane
                            const int end = __shfl(incl, l1, kWave);
                            take = end - used < take ? end - used : take;
                        }
                        const uint64_t upto = __ballot(excl < used + take) & nz;  // lanes before the take's end
                        ptup += __popcll(from & upto);
                    }
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
                            if constexpr (XF) {
                                const int32_t i3 = __shfl(iq3_l, lo, kWave), qp = __shfl(qpk_l, lo, kWave);
                                if (pos >= pend && pos < pend + take) {
                                    buf[k] = (uint64_t)j1 | ((uint64_t)j2 << 3) | ((uint64_t)j3 << 6) |
                                             ((uint64_t)(start + lo) << 9) | ((uint64_t)i3 << 33);
                                    qbuf[k] = qp;
                                }
                            } else {
                                const uint64_t g1 = (uint64_t)(iq1 * NB + j1);
                                const uint64_t g2 = (uint64_t)((start + lo) * NB + j2);
                                if (pos >= pend && pos < pend + take) buf[k] = g1 | (g2 << 24) | ((uint64_t)j3 << 48);
                            }
                        }
                    }
                    pend += take;
                    used += take;
                    if (pend == kBU || (XF && ptup == kXTB) || (last && pend > 0)) {
                        if (FORM == 0 && !folded) fold_unit();
                        if constexpr (FORM == 1)
                            tbm_batch<MAXT, false>(buf, pend, g0, type, fsp + fr * n_kblk * 4 * kWave * 3, omega,
                                                   evec32, occ, tm, groups, flag, a,
                                                   reinterpret_cast<const uint4*>(sroots), sA[wave], sQ[wave], accg,
                                                   accw, dl, 0.0, nullptr);
                        else if constexpr (FORM == 0)
                            tb_batch<MAXT, false, kBR, kFusedTB, true>(buf, pend, g0, type, fw, omega, evec, occ, bt,
                                                                       ft.fgroups, flag, a, sroots, sA[wave],
                                                                       sQ[wave], accg, accw, dl, 0.0, nullptr);
                        else
                            tbx_batch<MAXT, X32>(buf, qbuf, pend, g0, type, iq1, sF, omega, evec, evec32, ft.occt, bt,
                                            ft.pgroups, ft.n_pgroups, a, sroots, sA[wave], &sQ[wave][0][0], accg,
                                            accw);
                        pend = 0;
                        ptup = 0;
                        // the next batch writes every slot it reads; clearing them
                        // keeps the old records out of registers across the batch
#pragma unroll
                        for (int k = 0; k < kBR; ++k) {
                            buf[k] = 0;
                            qbuf[k] = 0;
                        }
                    }
                } while (used < total);
                if (last) break;
            }
            }  // live
        }
        double* out = partial + u * (2 * a.n_T);
        if constexpr (XF) {
            // the unit's sums: each wave's, then the four in wave order
#pragma unroll
            for (int it = 0; it < MAXT; ++it) {
                const double sg = wave_sum(accg[it]);
                const double sw = wave_sum(accw[it]);
                if (lane == 0) {
                    sRed[wave][it] = sg;
                    sRed[wave][MAXT + it] = sw;
                }
            }
            if (lane == 0) {
                sCnt[wave][0] = kept;
                sCnt[wave][1] = ntup;
            }
            __syncthreads();
            if (threadIdx.x < (unsigned)a.n_T) {
                const int it = threadIdx.x;
                double sg = 0.0, sw = 0.0;
                for (int wv = 0; wv < kWavesPerBlock; ++wv) {
                    sg += sRed[wv][it];
                    sw += sRed[wv][MAXT + it];
                }
                out[it] = sg;
                out[a.n_T + it] = sw;
            }
            if (threadIdx.x == 0) {
                int64_t kk = 0, tt = 0;
                for (int wv = 0; wv < kWavesPerBlock; ++wv) {
                    kk += sCnt[wv][0];
                    tt += sCnt[wv][1];
                }
                unit_kept[u] = kk;
                unit_tup[u] = tt;
            }
            __syncthreads();
        } else {
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
}

// parts[b] = sum of block b's slice of v[0..n) (slices of ceil(n / blocks)); a
// second k_sum_i64 over the parts gives the total (integer sums are exact in any
// order).
__global__ void k_sum_i64_parts(const int64_t* __restrict__ v, int64_t n, int64_t* __restrict__ parts) {
    __shared__ int64_t red[kBlock];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    int64_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
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
