// Tuple-batched four-phonon rate kernel (branch-batched contraction).
// Included once, by fp_lib.hip, after fp_kernels.h.
//
// All listed processes of one (lambda, q', q'') tuple share the phases
// ph_k = exp(2 pi i (Q1.A_k + Q2.B_k)/L) of every phase key k, so the
// phase-weighted force constants
//   A_g[c](tuple) = sum_{k in group g} ph_k(tuple) phit_k[c]     (c = beta gamma delta)
// are formed once per tuple and partner-atom group g, and each process only
// contracts them with its partner eigenvectors:
//   V = sum_g sum_{beta gamma delta} A_g[beta gamma delta] eps1(b_g)_beta eps2(c_g)_gamma eps3(d_g)_delta.
// Over a block of tuples, A_g is a complex matrix product (27 components x
// tuples, K = the group's phase keys) and runs on FP64 MFMA
// (v_mfma_f64_16x16x4f64); the per-process contraction (39 complex MACs per
// group) runs on the VALU.  The two pipes overlap across the waves of a SIMD.
//
// Work unit: 128 consecutive records of one row (two per lane).  Records of a
// tuple are contiguous when lists come from the library's enumerator; the
// kernel finds tuple boundaries itself (a change of (q', q'') between
// consecutive records), so any record order is correct, only slower.  Tuples
// are staged 32 at a time in LDS.
#pragma once

namespace fpk {

constexpr int kBU = 128;            // records per unit
constexpr int kBR = kBU / kWave;    // records per lane
constexpr int kTB = 32;             // tuples staged per batch
constexpr int kMaxKs = 4;           // K-steps of four keys per partner group (groups hold <= 16 keys)
constexpr int kStageTerms = 512;    // key tables up to this size are staged in LDS

// Dynamic LDS of the tuple-batched kernels: the root table (L entries), then the
// key table (8 int32 per phase key) when it has at most kStageTerms keys.
inline size_t tb_dyn_lds(int32_t L, int64_t n_keys) {
    return (size_t)L * sizeof(double2) + (n_keys <= kStageTerms ? (size_t)n_keys * 8 * sizeof(int32_t) : 0);
}

// Copy the root table (and the key table when it fits) into the block's
// dynamic LDS; returns the key table to read, staged or global.
__device__ inline const int32_t* tb_stage_terms(void* at, const int32_t* __restrict__ tmeta, int32_t n_keys) {
    if (n_keys > kStageTerms) return tmeta;
    int32_t* stm = reinterpret_cast<int32_t*>(at);
    for (int i = threadIdx.x; i < n_keys * 8; i += kBlock) stm[i] = tmeta[i];
    return stm;
}

__device__ inline const int32_t* tb_stage(double2* sroots, const double2* __restrict__ roots, int32_t L,
                                          const int32_t* __restrict__ tmeta, int32_t n_keys) {
    for (int i = threadIdx.x; i < L; i += kBlock) sroots[i] = roots[i];
    return tb_stage_terms(sroots + L, tmeta, n_keys);
}


// One batch of up to 128 consecutive records of one row (two per lane, record
// k * 64 + lane in rec[k]; `count` valid): decode, find the (q', q'') tuples,
// build A_g per tuple and partner group on FP64 MFMA, contract per process on
// the VALU, weight in FP64.  Adds this lane's Gamma and WP terms into
// accg/accw; with GRAD it also writes h_p = c_p conj(V_p) to hout[k * 64 + lane]
// and the record's decoding (last partner, packed signed wavevectors) to dout
// for the valid records, c_p = 2 pref w G / prod(omega) sum_T dl[T] occ_T.
// g0, type and count are wave-uniform; A and Qs are this wave's LDS staging.
// FOLD (the fused path, where every record of the batch shares q'): `groups`
// are the fused groups over B-keys, `tmeta` the B-key table (B at [4..6]), and
// `phit_row` this wave's folded table of the unit, already in the MFMA
// A-operand layout (K-step, component tile, lane), so the per-tuple phase is
// exp(2 pi i Q2.B / L) alone.
template <int MAXT, bool GRAD, int BR = kBR, int TB = kTB, bool FOLD = false>
__device__ inline void tb_batch(const uint64_t (&rec)[BR], int count, int32_t g0, int type,
                                const double2* __restrict__ phit_row, const double* __restrict__ omega,
                                const double2* __restrict__ evec, const double* __restrict__ occ,
                                const int32_t* __restrict__ tmeta, const int32_t* __restrict__ groups,
                                int* __restrict__ flag, const RatesArgs& a, const double2* sroots, double2 (*A)[27],
                                int32_t (*Qs)[2], double (&accg)[MAXT], double (&accw)[MAXT], const double (&dl)[MAXT],
                                double pref, double2* __restrict__ hout, uint4* __restrict__ dout = nullptr) {
    const int lane = threadIdx.x & (kWave - 1);
    const int li = lane & 15, lk = lane >> 4;
    const ModeGeom& geo = a.geo;
    const int nb = geo.nb;
    int s1, s2, s3;
    type_signs(type, s1, s2, s3);
    const double c1 = s1 > 0 ? 1.0 : -1.0;
    const double c2 = s2 > 0 ? 1.0 : -1.0;
    const double c3 = s3 > 0 ? 1.0 : -1.0;
    const int32_t iq0 = g0 / nb;
    const int32_t c00 = iq0 / (geo.N1 * geo.N2), c01 = (iq0 / geo.N2) % geo.N1, c02 = iq0 % geo.N2;
    const double w0 = omega[g0];

    // ---- records, tuple boundaries and slots
    Proc pr[BR];
    bool have[BR], first[BR];
    int slot[BR];
    uint64_t prev_last = ~0ull;
    int base = 0;
#pragma unroll
    for (int k = 0; k < BR; ++k) {
        const int idx = k * kWave + lane;
        have[k] = idx < count;
        pr[k] = setup_proc<4>(have[k], rec[k], type, s1, s2, s3, g0, c00, c01, c02, w0, geo, omega, a.n_modes,
                              flag, a.br);
        const uint64_t key = have[k] ? (((uint64_t)mode_q(pr[k].g1, geo) << 32) | (uint64_t)mode_q(pr[k].g2, geo))
                                     : ~0ull;
        uint64_t up = __shfl(key, (lane + kWave - 1) & (kWave - 1), kWave);
        if (lane == 0) up = prev_last;
        first[k] = have[k] && key != up;
        const uint64_t mask = __ballot(first[k]);
        const uint64_t le = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
        slot[k] = base + __popcll(mask & le) - 1;
        base += __popcll(mask);
        prev_last = __shfl(key, kWave - 1, kWave);
    }
    const int n_tup = __builtin_amdgcn_readfirstlane(base);

    double2 V[BR];
#pragma unroll
    for (int k = 0; k < BR; ++k) V[k] = make_double2(0.0, 0.0);
    for (int gi = 0; gi < a.n_groups; ++gi) {
        const int32_t* G = groups + gi * 8;
        const int32_t ab = G[0], ac = G[1], ad = G[2], t0 = G[3], t1 = G[4];
        const int n_ks = (t1 - t0 + 3) >> 2;  // <= kMaxKs: groups hold at most 16 keys
        // this group's force constants and phase vectors for every K-step, one load
        double2 Fk[kMaxKs][2];
        bool kv[kMaxKs];
#pragma unroll
        for (int ks = 0; ks < kMaxKs; ++ks) {
            const int term = t0 + 4 * ks + lk;
            kv[ks] = ks < n_ks && term < t1;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const int comp = mt * 16 + li;
                if (FOLD)  // zero where the key or the component does not exist
                    Fk[ks][mt] = ks < n_ks ? phit_row[((int64_t)(G[5] + ks) * 2 + mt) * kWave + lane]
                                           : make_double2(0.0, 0.0);
                else
                    Fk[ks][mt] = (kv[ks] && comp < 27) ? phit_row[(int64_t)term * 27 + comp] : make_double2(0.0, 0.0);
            }
        }
        // with one record per lane, this group's partner eigenvector components are
        // loaded here, together with the force constants, so that one memory
        // round trip per group covers both
        double2 xs[BR][3], ys[BR][3], zs[BR][3];
        if (BR == 1) {
#pragma unroll
            for (int k = 0; k < BR; ++k) {
                const double2* e1 = evec + (int64_t)pr[k].g1 * nb + 3 * ab;
                const double2* e2 = evec + (int64_t)pr[k].g2 * nb + 3 * ac;
                const double2* e3 = evec + (int64_t)pr[k].gl * nb + 3 * ad;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    xs[k][q] = ld_eps(e1 + q, c1);
                    ys[k][q] = ld_eps(e2 + q, c2);
                    zs[k][q] = ld_eps(e3 + q, c3);
                }
            }
        }
        for (int tb = 0; tb < n_tup; tb += TB) {
            const int nbt = n_tup - tb < TB ? n_tup - tb : TB;
            // tuple wavevectors of this batch, written by each tuple's first record
#pragma unroll
            for (int k = 0; k < BR; ++k) {
                const int s = slot[k] - tb;
                if (first[k] && s >= 0 && s < TB) {
                    Qs[s][0] = pr[k].Q10 | (pr[k].Q11 << 10) | (pr[k].Q12 << 20);
                    Qs[s][1] = pr[k].Q20 | (pr[k].Q21 << 10) | (pr[k].Q22 << 20);
                }
            }
            lds_fence();
            // A_g for the batch on MFMA: 2 component tiles x (1 or 2) tuple tiles,
            // one tuple tile at a time, K = the group's terms (at most 16), four
            // at a time.  The group's force constants and phase vectors were
            // loaded once for all its K-steps.  Complex products take three real
            // MFMAs (Karatsuba):
            //   k1 = (Fr + Fi) pr,  k2 = Fr (pi - pr),  k3 = Fi (pr + pi),
            //   Re = k1 - k3,  Im = k1 + k2.
            // the contraction below waits on gathers and LDS reads; it takes issue
            // priority over this MFMA phase, which another wave of the SIMD can
            // then fill
            __builtin_amdgcn_s_setprio(0);
            const int n_nt = (nbt + 15) >> 4;  // <= TB / 16
            for (int nt = 0; nt < n_nt; ++nt) {
                const int tj = nt * 16 + li;
                const bool tval = tj < nbt;
                int32_t qv[6];
                {
                    const int32_t qa = Qs[tval ? tj : 0][0], qb = Qs[tval ? tj : 0][1];
                    qv[0] = qa & 1023;
                    qv[1] = (qa >> 10) & 1023;
                    qv[2] = (qa >> 20) & 1023;
                    qv[3] = qb & 1023;
                    qv[4] = (qb >> 10) & 1023;
                    qv[5] = (qb >> 20) & 1023;
                }
                d4 k1[2], k2[2], k3[2];  // [component tile]
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) k1[mt] = k2[mt] = k3[mt] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < kMaxKs; ++ks) {
                    if (ks >= n_ks) break;
                    double2 ph = make_double2(0.0, 0.0);
                    if (kv[ks] && tval) {
                        uint32_t kk = 0;
                        const int32_t* tmp = tmeta + (t0 + 4 * ks + lk) * 8;
#pragma unroll
                        for (int d = FOLD ? 3 : 0; d < 6; ++d) kk += (uint32_t)(qv[d] * tmp[1 + d]);
                        ph = sroots[mod_l(kk, geo.L, geo.magic)];
                    }
                    const double pd = ph.y - ph.x, ps = ph.x + ph.y;
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        const double2 F = Fk[ks][mt];
                        k1[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.x + F.y, ph.x, k1[mt], 0, 0, 0);
                        k2[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.x, pd, k2[mt], 0, 0, 0);
                        k3[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.y, ps, k3[mt], 0, 0, 0);
                    }
                }
                // D[i = 4r + lk][j = li]: component mt*16 + 4r + lk of tuple nt*16 + li
                if (tval) {
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int cc = mt * 16 + 4 * r + lk;
                            if (cc < 27) A[tj][cc] = make_double2(k1[mt][r] - k3[mt][r], k1[mt][r] + k2[mt][r]);
                        }
                }
            }
            lds_fence();
            __builtin_amdgcn_s_setprio(3);
            // per-process contraction with this group's partner eigenvectors, one
            // record at a time (no hoisting of later records' gathers)
#pragma unroll
            for (int k = 0; k < BR; ++k) {
                const int s = slot[k] - tb;
                if (have[k] && s >= 0 && s < nbt) {
                    double2 x[3], y[3], z[3];
                    if (BR == 1) {
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            x[q] = xs[k][q];
                            y[q] = ys[k][q];
                            z[q] = zs[k][q];
                        }
                    } else {
                        const double2* e1 = evec + (int64_t)pr[k].g1 * nb + 3 * ab;
                        const double2* e2 = evec + (int64_t)pr[k].g2 * nb + 3 * ac;
                        const double2* e3 = evec + (int64_t)pr[k].gl * nb + 3 * ad;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            x[q] = ld_eps(e1 + q, c1);
                            y[q] = ld_eps(e2 + q, c2);
                            z[q] = ld_eps(e3 + q, c3);
                        }
                    }
                    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        double2 ub = make_double2(0.0, 0.0);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double2 vc = make_double2(0.0, 0.0);
#pragma unroll
                            for (int d = 0; d < 3; ++d) vc = cfma(vc, A[s][(b * 3 + c) * 3 + d], z[d]);
                            ub = cfma(ub, vc, y[c]);
                            // three LDS reads per step: hoisting all 27 would spill
                            __builtin_amdgcn_sched_barrier(0);
                        }
                        acc = cfma(acc, ub, x[b]);
                    }
                    V[k].x += acc.x;
                    V[k].y += acc.y;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            lds_fence();
        }
    }

    // ---- weights and occupations (FP64)
#pragma unroll
    for (int k = 0; k < BR; ++k) {
        const double V2 = V[k].x * V[k].x + V[k].y * V[k].y;
        double cw = 0.0;
#pragma unroll
        for (int it = 0; it < MAXT; ++it) {
            if (it < a.n_T) {
                const double* n = occ + (int64_t)it * a.n_modes;
                const double n1 = n[pr[k].g1], n2 = n[pr[k].g2], nl = n[pr[k].gl];
                double oc;
                if (type == 2)
                    oc = n1 * n2 * (1.0 + nl) - (1.0 + n1) * (1.0 + n2) * nl;
                else if (type == 3)
                    oc = n1 * (1.0 + n2) * (1.0 + nl) - (1.0 + n1) * n2 * nl;
                else
                    oc = (1.0 + n1) * (1.0 + n2) * (1.0 + nl) - n1 * n2 * nl;
                const double xw = pr[k].base * oc;
                accw[it] += xw;
                accg[it] += xw * V2;
                cw += dl[it] * oc;
            }
        }
        if (GRAD && have[k]) {
            cw *= 2.0 * pref * pr[k].base;
            hout[k * kWave + lane] = make_double2(cw * V[k].x, -cw * V[k].y);
            dout[k * kWave + lane] = make_uint4((uint32_t)pr[k].gl,
                                                (uint32_t)(pr[k].Q10 | (pr[k].Q11 << 10) | (pr[k].Q12 << 20)),
                                                (uint32_t)(pr[k].Q20 | (pr[k].Q21 << 10) | (pr[k].Q22 << 20)), 0u);
        }
    }
}

// GRAD = true: the first half of the adjoint.  Instead of the rate partials,
// write h_p = c_p conj(V_p) for every record, with c_p = 2 pref w G occ-weighted
// by dL/dGamma of the row (sum over temperatures), to hbuf[hbase + record].
// BR records per lane (units of 64 BR records), batches of TB tuples, at least
// OCC resident blocks per CU.  The root table is dynamic LDS of L entries.
template <int MAXT, bool GRAD, int BR = kBR, int TB = kTB, int OCC = 2>
__global__ __launch_bounds__(kBlock, OCC) void k_rates4b(FP_RATES_PARAMS, const double* __restrict__ dldg,
                                                                      double pref, double2* __restrict__ hbuf,
                                                                      uint4* __restrict__ hdec) {
    extern __shared__ double2 sroots[];
    __shared__ double2 sA[kWavesPerBlock][TB][27];
    __shared__ int32_t sQ[kWavesPerBlock][TB][2];
    const int32_t* tm = tb_stage(sroots, roots, a.geo.L, tmeta, a.n_keys);
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcd;
    const int64_t per_xcd = (a.n_units + kXcd - 1) / kXcd;
    const int64_t u_beg = xcd * per_xcd;
    const int64_t u_end = u_beg + per_xcd < a.n_units ? u_beg + per_xcd : a.n_units;
    const int64_t wstride = (int64_t)(gridDim.x / kXcd) * kWavesPerBlock;

    for (int64_t u = u_beg + (int64_t)(blockIdx.x / kXcd) * kWavesPerBlock + wave; u < u_end; u += wstride) {
        const UnitDesc ud = units[u];
        const int32_t row = __builtin_amdgcn_readfirstlane(ud.row);
        const int32_t count = __builtin_amdgcn_readfirstlane(ud.count);
        double accg[MAXT], accw[MAXT];
#pragma unroll
        for (int it = 0; it < MAXT; ++it) accg[it] = accw[it] = 0.0;
        if (row >= 0 && count > 0) {
            const RowInfo ri = rows[row];
            const int32_t g0 = __builtin_amdgcn_readfirstlane(ri.mode);
            const int type = __builtin_amdgcn_readfirstlane(ri.type);
            uint64_t rec[BR];
#pragma unroll
            for (int k = 0; k < BR; ++k) {
                const int idx = k * kWave + lane;
                rec[k] = idx < count ? ri.rec[ud.start + idx] : 0;
            }
            double dl[MAXT];
#pragma unroll
            for (int it = 0; it < MAXT; ++it) dl[it] = (GRAD && it < a.n_T) ? dldg[(int64_t)it * a.n_modes + g0] : 0.0;
            tb_batch<MAXT, GRAD, BR, TB>(rec, count, g0, type, phit + (int64_t)row * a.n_keys * 27, omega, evec, occ, tm,
                                 groups, flag, a, sroots, sA[wave], sQ[wave], accg, accw, dl, pref,
                                 GRAD ? hbuf + ri.hbase + ud.start : nullptr, GRAD ? hdec + ri.hbase + ud.start : nullptr);
        }
        if (GRAD) continue;
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
    }
}

}  // namespace fpk
