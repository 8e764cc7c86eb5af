// Adjoint of the rates: d(sum_{lambda,T} dL/dGamma_lambda(T) Gamma_lambda(T)) / dPhi.
// Included once, by fp_lib.hip, after fp_kernels.h.
//
// Gamma is quadratic in the force constants, so for every listed process p
//   dL/dPhi_t^{a0 c} = sum_p c_p Re(conj(V_p) dV_p/dPhi_t^{a0 c}),
//   c_p = 2 pref sum_T dL/dGamma(T) w occ_T G / prod(omega),
//   dV_p/dPhi_t^{a0 c} = s_t e_lambda(a0_t)_{a0} exp(i q.C_t) ph_t(p) P_p[c],
// with s_t = eV/sqrt(prod M), ph_t(p) = exp(2 pi i (Q1.A_t + Q2.B_t)/L) and
// P_p[c] = eps1_beta eps2_gamma (eps3_delta) the partner product of term t's
// group.  Per row (fixed lambda) the process sum is a matrix product over the
// process dimension:
//   D_t[c] = sum_p H[t,p] P[p,c],   H[t,p] = c_p conj(V_p) ph_t(p),
// which runs on FP64 MFMA (v_mfma_f64_16x16x4f64: 16 terms x 16 components,
// K = 4 processes per instruction, the lanes carrying the process dimension).
// V is recomputed, never stored.  Each block owns a fixed set of chunks of
// records (one row per chunk) and keeps its D tiles in registers across a
// chunk; at the end of a chunk it folds them with e_lambda and exp(i q.C_t)
// into its own partial dPhi, written by exactly one lane per entry, so the
// result does not depend on timing.  A final kernel sums the block partials in
// block order.  k_grad serves order 3 (short lists); order 4 uses the two-pass
// tuple form below (k_rates4b in its GRAD mode, then k_grad4t).
#pragma once

namespace fpk {

constexpr int kSub = kBlock;  // processes staged per sub-chunk (one per thread)

// Matrix element of one process (the forward contraction, one process per lane).
template <int M>
__device__ inline double2 vertex_one(const Proc& pr, double c1, double c2, double c3, int nb,
                                     const double2* __restrict__ evec, const double2* __restrict__ phit_row,
                                     const int32_t* __restrict__ groups, int n_groups,
                                     const int32_t* __restrict__ tmeta, const double2* sroots, const ModeGeom& geo) {
    double2 V = make_double2(0.0, 0.0);
    for (int gi = 0; gi < n_groups; ++gi) {
        const int32_t* G = groups + gi * 8;
        const int32_t ab = G[0], ac = G[1], ad = G[2], t0 = G[3], t1 = G[4];
        if (M == 3) {
            double2 P[9];
            const double2* e1 = evec + (int64_t)pr.g1 * nb + 3 * ab;
            const double2* e2 = evec + (int64_t)pr.g2 * nb + 3 * ac;
            double2 x[3], y[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                x[k] = ld_eps(e1 + k, c1);
                y[k] = ld_eps(e2 + k, c2);
            }
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) P[b * 3 + c] = cmul(x[b], y[c]);
            for (int t = t0; t < t1; ++t) {
                const int32_t* tm = tmeta + t * 8;
                const double2* F = phit_row + (int64_t)t * 9;
                double2 s = make_double2(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < 9; ++c) s = cfma(s, F[c], P[c]);
                const uint32_t k = (uint32_t)(pr.Q10 * tm[1] + pr.Q11 * tm[2] + pr.Q12 * tm[3]);
                V = cfma(V, sroots[mod_l(k, geo.L, geo.magic)], s);
            }
        } else {
            double2 x[3], w[9];
            const double2* e1 = evec + (int64_t)pr.g1 * nb + 3 * ab;
            const double2* e2 = evec + (int64_t)pr.g2 * nb + 3 * ac;
            const double2* e3 = evec + (int64_t)pr.gl * nb + 3 * ad;
            double2 y[3], z[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                x[k] = ld_eps(e1 + k, c1);
                y[k] = ld_eps(e2 + k, c2);
                z[k] = ld_eps(e3 + k, c3);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) w[c * 3 + d] = cmul(y[c], z[d]);
            for (int t = t0; t < t1; ++t) {
                const int32_t* tm = tmeta + t * 8;
                const double2* F = phit_row + (int64_t)t * 27;
                double2 s = make_double2(0.0, 0.0);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    double2 uu = make_double2(0.0, 0.0);
#pragma unroll
                    for (int c = 0; c < 9; ++c) uu = cfma(uu, F[b * 9 + c], w[c]);
                    s = cfma(s, uu, x[b]);
                }
                const uint32_t k = (uint32_t)(pr.Q10 * tm[1] + pr.Q11 * tm[2] + pr.Q12 * tm[3] + pr.Q20 * tm[4] +
                                              pr.Q21 * tm[5] + pr.Q22 * tm[6]);
                V = cfma(V, sroots[mod_l(k, geo.L, geo.magic)], s);
            }
        }
    }
    return V;
}

struct GradArgs {
    int64_t n_units;   // chunk descriptors
    int64_t n_modes;
    int32_t n_terms, n_keys, n_groups, n_pairs;  // terms (partials), phase keys (tables)
    int32_t n_T;
    ModeGeom geo;
    Broad br;
    double pref;
    Temps dummy;
};

// Pair table entry: {group, first key, key count (<= 16), first component}.
#define FP_GRAD_PARAMS                                                                                           \
    const double* __restrict__ omega, const double2* __restrict__ evec, const double* __restrict__ occ,         \
        const double2* __restrict__ roots, const double2* __restrict__ phit, const int32_t* __restrict__ tmeta,    \
        const int32_t* __restrict__ tc, const int32_t* __restrict__ groups, const int32_t* __restrict__ pairs,   \
        const double* __restrict__ tscale, const RowInfo* __restrict__ rows, const UnitDesc* __restrict__ units, \
        const double* __restrict__ dldg, double* __restrict__ gpart, int* __restrict__ flag, GradArgs a

template <int M, int MAXT, int MAXP>
__global__ __launch_bounds__(kBlock, 1) void k_grad(FP_GRAD_PARAMS) {
    constexpr int NC = M == 3 ? 9 : 27;    // components after the mode's own index
    constexpr int NCOMP = 3 * NC;          // 3^m entries per term
    __shared__ double2 sroots[kMaxRoots];
    __shared__ double2 sh_h[kSub];
    __shared__ int32_t sh_q[kSub][2];
    __shared__ int32_t sh_g[kSub][3];
    for (int i = threadIdx.x; i < a.geo.L; i += kBlock) sroots[i] = roots[i];
    __syncthreads();

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const ModeGeom geo = a.geo;
    const int nb = geo.nb;
    double* __restrict__ mypart = gpart + (int64_t)blockIdx.x * a.n_terms * NCOMP;
    const int li = lane & 15;   // A row (term) / B column (component) / D column
    const int lk = lane >> 4;   // K index (process within a K-step) / D row block
    const int pass_size = kWavesPerBlock * MAXP;
    const int n_pass = (a.n_pairs + pass_size - 1) / pass_size;

    for (int64_t u = blockIdx.x; u < a.n_units; u += gridDim.x) {
        const UnitDesc ud = units[u];
        const int32_t row = __builtin_amdgcn_readfirstlane(ud.row);
        const int32_t count = __builtin_amdgcn_readfirstlane(ud.count);
        if (row < 0 || count <= 0) continue;
        const RowInfo ri = rows[row];
        const int32_t g0 = __builtin_amdgcn_readfirstlane(ri.mode);
        const int type = __builtin_amdgcn_readfirstlane(ri.type);
        int s1, s2, s3;
        type_signs(type, s1, s2, s3);
        const int sl = M == 3 ? s2 : s3;
        const double c1 = s1 > 0 ? 1.0 : -1.0;
        const double c2 = s2 > 0 ? 1.0 : -1.0;
        const double c3 = sl > 0 ? 1.0 : -1.0;
        const int32_t iq0 = g0 / nb;
        const int32_t c00 = iq0 / (geo.N1 * geo.N2), c01 = (iq0 / geo.N2) % geo.N1, c02 = iq0 % geo.N2;
        const double w0 = omega[g0];
        const double2* __restrict__ phit_row = phit + (int64_t)row * a.n_keys * NC;
        double dl[MAXT];
#pragma unroll
        for (int it = 0; it < MAXT; ++it) dl[it] = it < a.n_T ? dldg[(int64_t)it * a.n_modes + g0] : 0.0;

        for (int pass = 0; pass < n_pass; ++pass) {
            d4 Cr[MAXP], Ci[MAXP];
#pragma unroll
            for (int j = 0; j < MAXP; ++j) Cr[j] = Ci[j] = d4{0.0, 0.0, 0.0, 0.0};
            for (int sub = 0; sub < count; sub += kSub) {
                // ---- stage: recompute V for one process per thread
                {
                    const int idx = sub + tid;
                    const bool have = idx < count;
                    const uint64_t rec = have ? ri.rec[ud.start + idx] : 0;
                    const Proc pr = setup_proc<M>(have, rec, type, s1, s2, s3, g0, c00, c01, c02, w0, geo, omega,
                                                  a.n_modes, flag, a.br);
                    const double2 V = vertex_one<M>(pr, c1, c2, c3, nb, evec, phit_row, groups, a.n_groups, tmeta,
                                                    sroots, geo);
                    double cw = 0.0;
#pragma unroll
                    for (int it = 0; it < MAXT; ++it) {
                        if (it < a.n_T) {
                            const double* n = occ + (int64_t)it * a.n_modes;
                            const double n1 = n[pr.g1], nl = n[pr.gl];
                            double oc;
                            if (M == 3) {
                                oc = type == 0 ? n1 - nl : 1.0 + n1 + nl;
                            } else {
                                const double n2 = n[pr.g2];
                                if (type == 2)
                                    oc = n1 * n2 * (1.0 + nl) - (1.0 + n1) * (1.0 + n2) * nl;
                                else if (type == 3)
                                    oc = n1 * (1.0 + n2) * (1.0 + nl) - (1.0 + n1) * n2 * nl;
                                else
                                    oc = (1.0 + n1) * (1.0 + n2) * (1.0 + nl) - n1 * n2 * nl;
                            }
                            cw += dl[it] * oc;
                        }
                    }
                    cw *= 2.0 * a.pref * pr.base;
                    sh_h[tid] = make_double2(cw * V.x, -cw * V.y);
                    sh_q[tid][0] = pr.Q10 | (pr.Q11 << 10) | (pr.Q12 << 20);
                    sh_q[tid][1] = pr.Q20 | (pr.Q21 << 10) | (pr.Q22 << 20);
                    sh_g[tid][0] = pr.g1;
                    sh_g[tid][1] = pr.g2;
                    sh_g[tid][2] = pr.gl;
                }
                __syncthreads();
                // ---- D tiles: each wave owns pairs wave + 4 j (+ pass offset)
#pragma unroll
                for (int j = 0; j < MAXP; ++j) {
                    const int pi = pass * pass_size + j * kWavesPerBlock + wave;
                    if (pi < a.n_pairs) {
                        const int32_t* PP = pairs + pi * 4;
                        const int32_t gi = PP[0], tbeg = PP[1], tcnt = PP[2], cbeg = PP[3];
                        const int32_t* G = groups + gi * 8;
                        const int32_t ab = G[0], ac = G[1], ad = G[2];
                        // A role: term tbeg + li; B role: component cbeg + li
                        const bool aval = li < tcnt;
                        const int32_t* tm = tmeta + (tbeg + (aval ? li : 0)) * 8;
                        const int32_t A0 = tm[1], A1 = tm[2], A2 = tm[3], B0 = tm[4], B1 = tm[5], B2 = tm[6];
                        const int cc = cbeg + li;
                        const bool bval = cc < NC;
                        const int cs = bval ? cc : 0;
                        const int beta = M == 3 ? cs / 3 : cs / 9;
                        const int gam = M == 3 ? cs % 3 : (cs / 3) % 3;
                        const int del = cs % 3;
                        d4 cr = Cr[j], ci = Ci[j];
                        for (int ks = 0; ks < kSub / 4; ++ks) {
                            const int p = 4 * ks + lk;
                            const double2 h = sh_h[p];
                            const int32_t q1 = sh_q[p][0], q2 = sh_q[p][1];
                            const uint32_t kk = (uint32_t)((q1 & 1023) * A0 + ((q1 >> 10) & 1023) * A1 +
                                                           ((q1 >> 20) & 1023) * A2 + (q2 & 1023) * B0 +
                                                           ((q2 >> 10) & 1023) * B1 + ((q2 >> 20) & 1023) * B2);
                            double2 H = cmul(h, sroots[mod_l(kk, geo.L, geo.magic)]);
                            if (!aval) H = make_double2(0.0, 0.0);
                            const double2 xe = ld_eps(evec + (int64_t)sh_g[p][0] * nb + 3 * ab + beta, c1);
                            const double2 ye = ld_eps(evec + (int64_t)sh_g[p][1] * nb + 3 * ac + gam, c2);
                            double2 P = cmul(xe, ye);
                            if (M == 4) P = cmul(P, ld_eps(evec + (int64_t)sh_g[p][2] * nb + 3 * ad + del, c3));
                            if (!bval) P = make_double2(0.0, 0.0);
                            cr = __builtin_amdgcn_mfma_f64_16x16x4f64(H.x, P.x, cr, 0, 0, 0);
                            cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-H.y, P.y, cr, 0, 0, 0);
                            ci = __builtin_amdgcn_mfma_f64_16x16x4f64(H.x, P.y, ci, 0, 0, 0);
                            ci = __builtin_amdgcn_mfma_f64_16x16x4f64(H.y, P.x, ci, 0, 0, 0);
                        }
                        Cr[j] = cr;
                        Ci[j] = ci;
                    }
                }
                __syncthreads();
            }
            // ---- fold: dPhi_t[a0][c] += s_t Re(e_lambda(a0_t)_a0 exp(i q.C_t) D_t[c])
#pragma unroll
            for (int j = 0; j < MAXP; ++j) {
                const int pi = pass * pass_size + j * kWavesPerBlock + wave;
                if (pi < a.n_pairs) {
                    const int32_t* PP = pairs + pi * 4;
                    const int32_t tbeg = PP[1], tcnt = PP[2], cbeg = PP[3];
                    const int cc = cbeg + li;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int ti = 4 * r + lk;  // D row held in register r of this lane
                        if (ti < tcnt && cc < NC) {
                            // D belongs to a phase key: every term of the key takes it
                            const int key = tbeg + ti;
                            const int32_t k0 = tmeta[key * 8], k1 = k0 + tmeta[key * 8 + 7];
                            for (int32_t t = k0; t < k1; ++t) {
                                const int32_t* tt = tc + (int64_t)t * 4;
                                const uint32_t kq = (uint32_t)(c00 * tt[0] + c01 * tt[1] + c02 * tt[2]);
                                const double2 phq = sroots[mod_l(kq, geo.L, geo.magic)];
                                const double2 D = cmul(phq, make_double2(Cr[j][r], Ci[j][r]));
                                const double sc = tscale[t];
                                double* out = mypart + (int64_t)t * NCOMP + cc;
#pragma unroll
                                for (int al = 0; al < 3; ++al) {
                                    const double2 e = evec[(int64_t)g0 * nb + 3 * tt[3] + al];
                                    out[al * NC] += sc * (e.x * D.x - e.y * D.y);
                                }
                            }
                        }
                    }
                }
            }
        }
    }
}

// Second pass of the order-4 adjoint in tuple form.  All processes of a
// (lambda, q', q'') tuple share the phases ph_t, so per partner group g
//   D_t[c] = sum_p h_p ph_t(p) P_p[c] = sum_tau ph_t(tau) B_tau[c],
//   B_tau[c] = sum_{p in tau} h_p P_p[c],  h_p = c_p conj(V_p) (from the first pass).
// A wave owns one (chunk of a row, partner group) work item.  It walks the
// chunk 64 records at a time: stages each record's h_p and its 3 x 3 partner
// eigenvector components for the group in LDS (one gather per record and
// group), finds the tuples, and then each lane forms B for exactly the
// (tuple, component) entry that it feeds to the MFMA B-operand, while the
// A-operand carries ph_t(tau) for its (term, tuple) entry.  G = sum over tuples
// accumulates on FP64 MFMA (three real products per complex one); after the
// chunk it is folded with e_lambda and exp(i q.C_t) into the wave's own partial
// dPhi, so the final block-order reduction makes the result deterministic.
// Groups hold at most 16 phase keys: one 16-key A tile.
__global__ __launch_bounds__(kBlock, 2) void k_grad4t(const double2* __restrict__ evec, const double2* __restrict__ roots,
                                                     const int32_t* __restrict__ tmeta, const int32_t* __restrict__ tc,
                                                     const int32_t* __restrict__ groups,
                                                     const double* __restrict__ tscale,
                                                     const RowInfo* __restrict__ rows,
                                                     const UnitDesc* __restrict__ units,
                                                     const double2* __restrict__ hbuf,
                                                     const uint4* __restrict__ hdec, double* __restrict__ gpart,
                                                     int* __restrict__ flag, GradArgs a) {
    extern __shared__ double2 sroots[];  // L roots of unity (dynamic: sized by the launch)
    __shared__ double2 sU[kWavesPerBlock][kWave][3];  // h x_b per record
    __shared__ double2 sW[kWavesPerBlock][kWave][9];  // y_g z_d per record
    __shared__ int32_t sT[kWavesPerBlock][kWave + 1];  // first record of each tuple, then the end
    __shared__ int32_t sQ[kWavesPerBlock][kWave][2];
    for (int i = threadIdx.x; i < a.geo.L; i += kBlock) sroots[i] = roots[i];
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const ModeGeom geo = a.geo;
    const int nb = geo.nb;
    const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wave;  // this wave's partial
    const int64_t n_waves = (int64_t)gridDim.x * kWavesPerBlock;
    double* __restrict__ mypart = gpart + gw * a.n_terms * 81;
    double2(*U)[3] = sU[wave];
    double2(*W)[9] = sW[wave];
    int32_t* T = sT[wave];
    int32_t(*Qs)[2] = sQ[wave];
    const int64_t n_items = a.n_units * a.n_groups;

    for (int64_t item = gw; item < n_items; item += n_waves) {
        const int64_t chunk = item / a.n_groups;
        const int gi = (int)(item % a.n_groups);
        const UnitDesc ud = units[chunk];
        const int32_t row = __builtin_amdgcn_readfirstlane(ud.row);
        const int32_t count = __builtin_amdgcn_readfirstlane(ud.count);
        if (row < 0 || count <= 0) continue;
        const RowInfo ri = rows[row];
        const int32_t g0 = __builtin_amdgcn_readfirstlane(ri.mode);
        if (g0 < 0) continue;
        const int type = __builtin_amdgcn_readfirstlane(ri.type);
        int s1, s2, s3;
        type_signs(type, s1, s2, s3);
        const double c1 = s1 > 0 ? 1.0 : -1.0;
        const double c2 = s2 > 0 ? 1.0 : -1.0;
        const double c3 = s3 > 0 ? 1.0 : -1.0;
        const int32_t iq0 = g0 / nb;
        const int32_t c00 = iq0 / (geo.N1 * geo.N2), c01 = (iq0 / geo.N2) % geo.N1, c02 = iq0 % geo.N2;
        const int32_t* G = groups + gi * 8;
        const int32_t ab = G[0], ac = G[1], ad = G[2], t0 = G[3], t1 = G[4];
        // this lane's A-operand term and its phase vectors
        const int term = t0 + li;
        const bool tv = term < t1;
        int32_t tm[6];
        {
            const int32_t* tp = tmeta + (tv ? term : t0) * 8;
#pragma unroll
            for (int d = 0; d < 6; ++d) tm[d] = tp[1 + d];
        }
        d4 k1[2], k2[2], k3[2];  // [component tile]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) k1[mt] = k2[mt] = k3[mt] = d4{0.0, 0.0, 0.0, 0.0};

        for (int sub = 0; sub < count; sub += kWave) {
            const int n_here = count - sub < kWave ? count - sub : kWave;
            const int idx = sub + lane;
            const bool have = lane < n_here;
            const uint64_t rec = have ? ri.rec[ud.start + idx] : 0;
            // the first pass decoded the record (last partner closed by momentum,
            // signed wavevectors packed as the phase index needs them); a record it
            // found out of range has h = 0 and is read with the row's mode
            Proc pr;
            {
                const uint4 dv = have ? hdec[ri.hbase + ud.start + idx] : make_uint4((uint32_t)g0, 0u, 0u, 0u);
                pr.g1 = (int32_t)(rec & 0xFFFFFFu);
                pr.g2 = (int32_t)((rec >> 24) & 0xFFFFFFu);
                if (!have || pr.g1 >= a.n_modes || pr.g2 >= a.n_modes) pr.g1 = pr.g2 = g0;
                pr.gl = (int32_t)dv.x;
                pr.Q10 = (int32_t)dv.y;  // packed Q1 (10 bits per axis)
                pr.Q20 = (int32_t)dv.z;  // packed Q2
            }
            const uint64_t key = have ? (((uint64_t)mode_q(pr.g1, geo) << 32) | (uint64_t)mode_q(pr.g2, geo)) : ~0ull;
            const uint64_t up = __shfl(key, (lane + kWave - 1) & (kWave - 1), kWave);
            const bool first = have && (lane == 0 || key != up);
            const uint64_t mask = __ballot(first);
            const uint64_t le = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
            const int slot = __popcll(mask & le) - 1;
            const int n_tup = __builtin_amdgcn_readfirstlane(__popcll(mask));
            if (first) {
                T[slot] = lane;
                Qs[slot][0] = pr.Q10;
                Qs[slot][1] = pr.Q20;
            }
            if (lane == 0) T[n_tup] = n_here;
            // this lane's record: h_p x_b and y_g z_d for the group's partner atoms
            {
                const double2 h = have ? hbuf[ri.hbase + ud.start + idx] : make_double2(0.0, 0.0);
                const double2* e1 = evec + (int64_t)pr.g1 * nb + 3 * ab;
                const double2* e2 = evec + (int64_t)pr.g2 * nb + 3 * ac;
                const double2* e3 = evec + (int64_t)pr.gl * nb + 3 * ad;
                double2 y[3], z[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    U[lane][q] = cmul(h, ld_eps(e1 + q, c1));
                    y[q] = ld_eps(e2 + q, c2);
                    z[q] = ld_eps(e3 + q, c3);
                }
#pragma unroll
                for (int g = 0; g < 3; ++g)
#pragma unroll
                    for (int d = 0; d < 3; ++d) W[lane][g * 3 + d] = cmul(y[g], z[d]);
            }
            lds_fence();
            const int n_ks = (n_tup + 3) >> 2;
            for (int ks = 0; ks < n_ks; ++ks) {
                const int s = 4 * ks + lk;  // this lane's tuple (A column, B row)
                const bool sv = s < n_tup;
                // A-operand: ph_term(tuple)
                double2 ph = make_double2(0.0, 0.0);
                int r0 = 0, r1 = 0;
                if (sv) {
                    r0 = T[s];
                    r1 = T[s + 1];
                    if (tv) {
                        const int32_t qa = Qs[s][0], qb = Qs[s][1];
                        const uint32_t kk = (uint32_t)((qa & 1023) * tm[0] + ((qa >> 10) & 1023) * tm[1] +
                                                       ((qa >> 20) & 1023) * tm[2] + (qb & 1023) * tm[3] +
                                                       ((qb >> 10) & 1023) * tm[4] + ((qb >> 20) & 1023) * tm[5]);
                        ph = sroots[mod_l(kk, geo.L, geo.magic)];
                    }
                }
                const double pd_s = ph.x + ph.y;
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    // B-operand: B_tuple[c] for component c = 16 mt + li
                    const int c = mt * 16 + li;
                    double2 B = make_double2(0.0, 0.0);
                    // the tuple sums wait on LDS; they take issue priority over
                    // another wave's MFMAs
                    __builtin_amdgcn_s_setprio(3);
                    if (c < 27) {
                        const int b = c / 9, gd = c % 9;
                        for (int r = r0; r < r1; ++r) B = cfma(B, U[r][b], W[r][gd]);
                    }
                    __builtin_amdgcn_s_setprio(0);
                    // G += ph B (Karatsuba: k1 = (Ar + Ai) Br, k2 = Ar (Bi - Br), k3 = Ai (Br + Bi))
                    k1[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pd_s, B.x, k1[mt], 0, 0, 0);
                    k2[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ph.x, B.y - B.x, k2[mt], 0, 0, 0);
                    k3[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ph.y, B.x + B.y, k3[mt], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            lds_fence();
        }
        // fold: dPhi_t[a0][c] += s_t Re(e_lambda(a0_t)_a0 exp(i q.C_t) D_t[c]); D row 4 r + lk, column li
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const int c = mt * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int key = t0 + 4 * r + lk;
                if (key < t1 && c < 27) {
                    // D belongs to a phase key: every term of the key takes it
                    const double2 D = make_double2(k1[mt][r] - k3[mt][r], k1[mt][r] + k2[mt][r]);
                    const int32_t kb = tmeta[key * 8], ke = kb + tmeta[key * 8 + 7];
                    for (int32_t t = kb; t < ke; ++t) {
                        const int32_t* tt = tc + (int64_t)t * 4;
                        const uint32_t kq = (uint32_t)(c00 * tt[0] + c01 * tt[1] + c02 * tt[2]);
                        const double2 Dq = cmul(sroots[mod_l(kq, geo.L, geo.magic)], D);
                        const double sc = tscale[t];
                        double* out = mypart + (int64_t)t * 81 + c;
#pragma unroll
                        for (int al = 0; al < 3; ++al) {
                            const double2 e = evec[(int64_t)g0 * nb + 3 * tt[3] + al];
                            out[al * 27] += sc * (e.x * Dq.x - e.y * Dq.y);
                        }
                    }
                }
            }
        }
    }
}

// First level of the partial-gradient reduction: out[s][i] = sum of
// gpart[b][i] over the parts b of slab s (kSlab consecutive parts, in order).
constexpr int kSlab = 32;
__global__ void k_grad_slab(const double* __restrict__ gpart, int64_t n_parts, int64_t n, double* __restrict__ out) {
    const int64_t n_slabs = (n_parts + kSlab - 1) / kSlab;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_slabs * n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sl = j / n, i = j % n;
        const int64_t b1 = (sl + 1) * kSlab < n_parts ? (sl + 1) * kSlab : n_parts;
        double s = 0.0;
        for (int64_t b = sl * kSlab; b < b1; ++b) s += gpart[b * n + i];
        out[j] = s;
    }
}

// dphi[perm[t]][k] (+)= sum_b gpart[b][t][k], summed in block order.
__global__ void k_grad_reduce(const double* __restrict__ gpart, int64_t n_blocks, int64_t n_terms, int32_t ncomp,
                              const int32_t* __restrict__ perm, int accumulate, double* __restrict__ dphi) {
    const int64_t n = n_terms * ncomp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t b = 0; b < n_blocks; ++b) s += gpart[b * n + i];
        const int64_t t = i / ncomp, k = i % ncomp;
        double* o = dphi + (int64_t)perm[t] * ncomp + k;
        *o = accumulate ? *o + s : s;
    }
}

}  // namespace fpk
