// Mixed-precision four-phonon rate kernel (FP_MIXED).
// Included once, by fp_lib.hip, after fp_batched.h.
//
// Same tuple-batched formulation as k_rates4b, with the precision split as
// follows:
//   - phase-weighted force constants A_g[c](tuple) = sum_t ph_t phit_t[c] run on
//     bf16 MFMA (v_mfma_f32_16x16x32_bf16) with split-precision operands: each
//     FP64 operand is written as a sum of three bf16 numbers (x = h0 + h1 + h2,
//     residuals formed in FP64) and the six products h_a h_b with a + b <= 2 are
//     accumulated in FP32, which reproduces an FP32-accurate product;
//   - the phases are exact roots of unity taken from the FP64 table before the
//     split;
//   - the per-process eigenvector contraction runs in FP32;
//   - |V|^2 is formed in FP64, and the Gaussian, occupations, 1/prod(omega),
//     temperature loop and all accumulation of Gamma stay in FP64.
//
// The complex product is a real GEMM with K = (term, re/im part) and M =
// (component, re/im of the result):
//   Re A = sum_t (Fr pr - Fi pi),  Im A = sum_t (Fi pr + Fr pi),
// so row (c, 0) of the A-operand holds (Fr, -Fi) and row (c, 1) holds (Fi, Fr)
// against the B-operand column (pr, pi) of each tuple.  One K-step covers 16
// terms of a group; four M-tiles cover the 27 components.
#pragma once

namespace fpk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// float -> bf16 bit pattern, round to nearest even (finite inputs).
__device__ inline uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ inline double bf16_to_double(uint32_t b) { return (double)__uint_as_float(b << 16); }

// x ~= h[0] + h[1] + h[2] in bf16; each residual is formed in FP64.
__device__ inline void split3(double x, uint32_t h[3]) {
    double r = x;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        h[s] = bf16_bits((float)r);
        r -= bf16_to_double(h[s]);
    }
}

__device__ inline bf16x8 as_bf16x8(uint4 w) { return __builtin_bit_cast(bf16x8, w); }

// Split planes of the pre-contracted force constants, laid out as the MFMA
// A-operand wants them: for row r, K-block b (16 terms of one group), M-tile mt
// and lane l, three uint4 (one per split level) holding 8 bf16 for
// A[i = l % 16][k = 8 (l / 16) + v], v = 0..7, with i = 2 (c - 8 mt) + ri and
// k = 2 (term - first term of the block) + part.
__global__ void k_split_phit(int64_t total_rows, const double2* __restrict__ phit, const int32_t* __restrict__ groups,
                             const int32_t* __restrict__ kblk, int32_t n_kblk, int32_t n_keys, uint4* __restrict__ fsp) {
    const int64_t n = total_rows * n_kblk * 4 * kWave;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(x % kWave);
        const int mt = (int)((x / kWave) % 4);
        const int64_t rb = x / (4 * kWave);
        const int32_t b = (int32_t)(rb % n_kblk);
        const int64_t row = rb / n_kblk;
        const int32_t g = kblk[2 * b], ks = kblk[2 * b + 1];
        const int32_t t0 = groups[g * 8 + 3], t1 = groups[g * 8 + 4];
        const int i = lane & 15, kq = lane >> 4;
        const int comp = 8 * mt + (i >> 1), ri = i & 1;
        uint32_t w[3][4];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int t = t0 + 16 * ks + 4 * kq + (v >> 1);
            const int part = v & 1;
            double2 F = make_double2(0.0, 0.0);
            if (t < t1 && comp < 27) F = phit[((int64_t)row * n_keys + t) * 27 + comp];
            const double a = ri == 0 ? (part == 0 ? F.x : -F.y) : (part == 0 ? F.y : F.x);
            uint32_t h[3];
            split3(a, h);
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                if (v & 1)
                    w[s][v >> 1] |= h[s] << 16;
                else
                    w[s][v >> 1] = h[s];
            }
        }
        uint4* out = fsp + x * 3;
#pragma unroll
        for (int s = 0; s < 3; ++s) out[s] = make_uint4(w[s][0], w[s][1], w[s][2], w[s][3]);
    }
}

#define FP_RATES_MIXED_PARAMS                                                                                    \
    const double* __restrict__ omega, const float2* __restrict__ evec32, const double* __restrict__ occ,        \
        const double2* __restrict__ roots, const uint4* __restrict__ fsp, const int32_t* __restrict__ tmeta,    \
        const int32_t* __restrict__ groups, const RowInfo* __restrict__ rows, const UnitDesc* __restrict__ units, \
        double* __restrict__ partial, int* __restrict__ flag, RatesArgs a, int32_t n_kblk

__device__ inline float2 cfmaf(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}

__device__ inline float2 ld_eps32(const float2* __restrict__ e, float csign) {
    float2 v = *e;
    v.y *= csign;
    return v;
}

// One batch of up to 128 consecutive records of one row (record k * 64 + lane
// in rec[k]; `count` valid), in mixed precision: the phase-weighted force
// constants of each (q', q'') tuple on bf16 split MFMA with FP32 accumulation,
// the contraction in FP32, weights and sums in FP64.  Adds this lane's Gamma
// and WP terms into accg/accw; with GRAD it writes h_p = c_p conj(V_p) to
// hout[k * 64 + lane] for the valid records.  g0, type and count are
// wave-uniform; sroot, A and Qs are LDS (the root split table, this wave's
// staging).
template <int MAXT, bool GRAD>
__device__ inline void tbm_batch(const uint64_t (&rec)[kBR], int count, int32_t g0, int type,
                                 const uint4* __restrict__ fsp_row, const double* __restrict__ omega,
                                 const float2* __restrict__ evec32, const double* __restrict__ occ,
                                 const int32_t* __restrict__ tmeta, const int32_t* __restrict__ groups,
                                 int* __restrict__ flag, const RatesArgs& a, const uint4* sroot, float2 (*A)[27],
                                 int32_t (*Qs)[2], double (&accg)[MAXT], double (&accw)[MAXT],
                                 const double (&dl)[MAXT], double pref, double2* __restrict__ hout,
                                 uint4* __restrict__ dout = nullptr) {
    const int lane = threadIdx.x & (kWave - 1);
    const int li = lane & 15, lk = lane >> 4;
    const ModeGeom& geo = a.geo;
    const int nb = geo.nb;
    int s1, s2, s3;
    type_signs(type, s1, s2, s3);
    const float c1 = s1 > 0 ? 1.0f : -1.0f;
    const float c2 = s2 > 0 ? 1.0f : -1.0f;
    const float c3 = s3 > 0 ? 1.0f : -1.0f;
    const int32_t iq0 = g0 / nb;
    const int32_t c00 = iq0 / (geo.N1 * geo.N2), c01 = (iq0 / geo.N2) % geo.N1, c02 = iq0 % geo.N2;
    const double w0 = omega[g0];

    // ---- records, tuple boundaries and slots (as in the FP64 tuple-batched kernel)
    Proc pr[kBR];
    bool have[kBR], first[kBR];
    int slot[kBR];
    uint64_t prev_last = ~0ull;
    int base = 0;
#pragma unroll
    for (int k = 0; k < kBR; ++k) {
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

    float2 V[kBR];
#pragma unroll
    for (int k = 0; k < kBR; ++k) V[k] = make_float2(0.0f, 0.0f);
    for (int gi = 0; gi < a.n_groups; ++gi) {
        const int32_t* G = groups + gi * 8;
        const int32_t ab = G[0], ac = G[1], ad = G[2], t0 = G[3], t1 = G[4], kb0 = G[5];
        const int n_ks = (t1 - t0 + 15) >> 4;
        for (int tb = 0; tb < n_tup; tb += kTB) {
            const int nbt = n_tup - tb < kTB ? n_tup - tb : kTB;
#pragma unroll
            for (int k = 0; k < kBR; ++k) {
                const int s = slot[k] - tb;
                if (first[k] && s >= 0 && s < kTB) {
                    Qs[s][0] = pr[k].Q10 | (pr[k].Q11 << 10) | (pr[k].Q12 << 20);
                    Qs[s][1] = pr[k].Q20 | (pr[k].Q21 << 10) | (pr[k].Q22 << 20);
                }
            }
            lds_fence();
            const bool two = nbt > 16;
            int32_t qv[2][6];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int tj = nt * 16 + li;
                const int32_t qa = Qs[tj < nbt ? tj : 0][0], qb = Qs[tj < nbt ? tj : 0][1];
                qv[nt][0] = qa & 1023;
                qv[nt][1] = (qa >> 10) & 1023;
                qv[nt][2] = (qa >> 20) & 1023;
                qv[nt][3] = qb & 1023;
                qv[nt][4] = (qb >> 10) & 1023;
                qv[nt][5] = (qb >> 20) & 1023;
            }
            f4v acc[2][4];  // [tuple tile][component tile]
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) acc[nt][mt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks = 0; ks < n_ks; ++ks) {
                // A-operand split planes of this K-block, all four M-tiles
                uint4 Aw[4][3];
                const uint4* src = fsp_row + ((int64_t)(kb0 + ks) * 4 * kWave + lane) * 3;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int s = 0; s < 3; ++s) Aw[mt][s] = src[mt * kWave * 3 + s];
                // the four terms of this lane's K-slice
                int32_t tm[4][6];
                bool tv[4];
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    const int t = t0 + 16 * ks + 4 * lk + tt;
                    tv[tt] = t < t1;
                    const int32_t* tp = tmeta + (tv[tt] ? t : t0) * 8;
#pragma unroll
                    for (int d = 0; d < 6; ++d) tm[tt][d] = tp[1 + d];
                }
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    if (nt == 1 && !two) break;
                    const bool tval = nt * 16 + li < nbt;
                    uint4 bw[4];
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        bw[tt] = make_uint4(0u, 0u, 0u, 0u);
                        if (tv[tt] && tval) {
                            uint32_t kk = 0;
#pragma unroll
                            for (int d = 0; d < 6; ++d) kk += (uint32_t)(qv[nt][d] * tm[tt][d]);
                            bw[tt] = sroot[mod_l(kk, geo.L, geo.magic)];
                        }
                    }
                    const bf16x8 B0 = as_bf16x8(make_uint4(bw[0].x, bw[1].x, bw[2].x, bw[3].x));
                    const bf16x8 B1 = as_bf16x8(make_uint4(bw[0].y, bw[1].y, bw[2].y, bw[3].y));
                    const bf16x8 B2 = as_bf16x8(make_uint4(bw[0].z, bw[1].z, bw[2].z, bw[3].z));
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        const bf16x8 A0 = as_bf16x8(Aw[mt][0]), A1 = as_bf16x8(Aw[mt][1]),
                                     A2 = as_bf16x8(Aw[mt][2]);
                        f4v c = acc[nt][mt];
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2, B0, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B1, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B2, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B0, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B1, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B0, c, 0, 0, 0);
                        acc[nt][mt] = c;
                    }
                }
            }
            // D[i = 4 lk + r][j = li]: component 8 mt + 2 lk + r / 2, part r % 2, tuple 16 nt + li
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int tj = nt * 16 + li;
                if (tj < nbt) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        const int cc = 8 * mt + 2 * lk;
                        if (cc < 27) A[tj][cc] = make_float2(acc[nt][mt][0], acc[nt][mt][1]);
                        if (cc + 1 < 27) A[tj][cc + 1] = make_float2(acc[nt][mt][2], acc[nt][mt][3]);
                    }
                }
            }
            lds_fence();
#pragma unroll
            for (int k = 0; k < kBR; ++k) {
                const int s = slot[k] - tb;
                if (have[k] && s >= 0 && s < nbt) {
                    const float2* e1 = evec32 + (int64_t)pr[k].g1 * nb + 3 * ab;
                    const float2* e2 = evec32 + (int64_t)pr[k].g2 * nb + 3 * ac;
                    const float2* e3 = evec32 + (int64_t)pr[k].gl * nb + 3 * ad;
                    float2 x[3], y[3], z[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        x[q] = ld_eps32(e1 + q, c1);
                        y[q] = ld_eps32(e2 + q, c2);
                        z[q] = ld_eps32(e3 + q, c3);
                    }
                    float2 accv = make_float2(0.0f, 0.0f);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        float2 ub = make_float2(0.0f, 0.0f);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            float2 vc = make_float2(0.0f, 0.0f);
#pragma unroll
                            for (int d = 0; d < 3; ++d) vc = cfmaf(vc, A[s][(b * 3 + c) * 3 + d], z[d]);
                            ub = cfmaf(ub, vc, y[c]);
                        }
                        accv = cfmaf(accv, ub, x[b]);
                    }
                    V[k].x += accv.x;
                    V[k].y += accv.y;
                }
            }
            lds_fence();
        }
    }

    // ---- weights and occupations (FP64)
#pragma unroll
    for (int k = 0; k < kBR; ++k) {
        const double vx = V[k].x, vy = V[k].y;
        const double V2 = vx * vx + vy * vy;
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
            hout[k * kWave + lane] = make_double2(cw * vx, -cw * vy);
            dout[k * kWave + lane] = make_uint4((uint32_t)pr[k].gl,
                                                (uint32_t)(pr[k].Q10 | (pr[k].Q11 << 10) | (pr[k].Q12 << 20)),
                                                (uint32_t)(pr[k].Q20 | (pr[k].Q21 << 10) | (pr[k].Q22 << 20)), 0u);
        }
    }
}

// Root table as three bf16 splits of (Re, Im): word s of entry i = split s.
__device__ inline void tbm_roots(uint4* sroot, const double2* __restrict__ roots, int32_t L) {
    for (int i = threadIdx.x; i < L; i += kBlock) {
        const double2 r = roots[i];
        uint32_t hr[3], hi[3];
        split3(r.x, hr);
        split3(r.y, hi);
        sroot[i] = make_uint4(hr[0] | (hi[0] << 16), hr[1] | (hi[1] << 16), hr[2] | (hi[2] << 16), 0u);
    }
}

// GRAD = true: first pass of the mixed-precision adjoint.  Instead of the rate
// partials, write h_p = c_p conj(V_p) in FP64 for every record (V from the
// mixed-precision contraction), as the FP64 tuple-batched kernel does.
template <int MAXT, bool GRAD>
__global__ __launch_bounds__(kBlock, 2) void k_rates4m(FP_RATES_MIXED_PARAMS, const double* __restrict__ dldg,
                                                      double pref, double2* __restrict__ hbuf,
                                                      uint4* __restrict__ hdec) {
    __shared__ uint4 sroot[kMaxRoots];  // word s = bf16 split s of (Re, Im) of the root
    __shared__ float2 sA[kWavesPerBlock][kTB][27];
    __shared__ int32_t sQ[kWavesPerBlock][kTB][2];
    tbm_roots(sroot, roots, a.geo.L);
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcd;
    const int64_t per_xcd = (a.n_units + kXcd - 1) / kXcd;
    const int64_t u_beg = xcd * per_xcd;
    const int64_t u_end = u_beg + per_xcd < a.n_units ? u_beg + per_xcd : a.n_units;
    const int64_t wstride = (int64_t)(gridDim.x / kXcd) * kWavesPerBlock;
    float2(*A)[27] = sA[wave];
    int32_t(*Qs)[2] = sQ[wave];

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
            uint64_t rec[kBR];
#pragma unroll
            for (int k = 0; k < kBR; ++k) {
                const int idx = k * kWave + lane;
                rec[k] = idx < count ? ri.rec[ud.start + idx] : 0;
            }
            double dl[MAXT];
#pragma unroll
            for (int it = 0; it < MAXT; ++it) dl[it] = (GRAD && it < a.n_T) ? dldg[(int64_t)it * a.n_modes + g0] : 0.0;
            tbm_batch<MAXT, GRAD>(rec, count, g0, type, fsp + (int64_t)row * n_kblk * 4 * kWave * 3, omega, evec32, occ,
                                  tmeta, groups, flag, a, sroot, A, Qs, accg, accw, dl, pref,
                                  GRAD ? hbuf + ri.hbase + ud.start : nullptr,
                                  GRAD ? hdec + ri.hbase + ud.start : nullptr);
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
