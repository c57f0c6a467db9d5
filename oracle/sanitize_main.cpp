// sanitize_main.cpp -- a host driver that runs every exported routine of the
// FP64 oracle once on small inputs, for a build under AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py builds it with
// g++ and fails on any report).  TEST INFRASTRUCTURE ONLY, like the oracle.
//
// Two contexts: a homogeneous medium with a von Mises-Fisher source and the
// paper's angular sensor response, and a layered medium (simplified-Liu
// mixture in some layers) with a uniform-cone source and a sector tilt.
// Each is driven through the sampler (plain, joint and single-vertex
// Langevin), the proposals from continuous draws, the density, the
// gradients, both anchor quadratures and the analog tracer.
#include "rjoracle.cpp"

#include <cstdio>

namespace {

void path3(double D, double* v) {
    // source, one vertex off the axis, end point on the sensor facing it
    v[0] = v[1] = v[2] = 0.0;
    v[3] = 0.4; v[4] = -0.2; v[5] = 0.5 * D;
    v[6] = 0.0; v[7] = 0.0; v[8] = D - 0.165;
}

int exercise(void* h, int cap, int n_targets, double D) {
    // sampler runs: plain, joint Langevin, single-vertex Langevin
    for (int sampler = 0; sampler <= 2; ++sampler) {
        const int C = 6;
        uint64_t ip[8] = {7, 0, 5, 60, 5, 3, 1u << 31, (uint64_t)sampler};
        double dp[3] = {0.5, 20.0, sampler == 1 ? 0.01 : 0.2};
        std::vector<int> ids(C), tgt(C), n(C, 3);
        std::vector<double> v((size_t)C * cap * 3, 0.0), stats((size_t)C * 16, 0.0), trace((size_t)C * 60 * 5);
        for (int c = 0; c < C; ++c) {
            ids[c] = c;
            tgt[c] = c % n_targets;
            path3(D, &v[(size_t)c * cap * 3]);
        }
        orc_run(h, ip, dp, C, ids.data(), tgt.data(), n.data(), v.data(), stats.data(), trace.data(), 2);
        int nn = n[0];
        double rec[5];
        int np_ = 0;
        std::vector<double> prop((size_t)(cap + 1) * 3);
        orc_step(h, ip, dp, 0, tgt[0], &nn, v.data(), rec, &np_, prop.data());
    }
    // proposals from continuous draws
    uint64_t ip[8] = {7, 0, 0, 1, 5, 3, 1u << 31, 2};
    double dp[3] = {0.5, 20.0, 0.2};
    double v[9], y[12], u[8] = {0.3, 0.6, 0.2, 0.7, 0.4, 0.55, 0.25, 0.8};
    path3(D, v);
    int ny = 0, mv = 0;
    double s = 0;
    s += orc_propose(h, ip, dp, 0, 0, 3, v, 1, u, &ny, y, &mv);
    s += orc_propose(h, ip, dp, 0, 0, 3, v, 2, u, &ny, y, &mv);
    s += orc_propose(h, ip, dp, 0, 1, 3, v, 0, u, &ny, y, &mv);
    s += orc_propose(h, ip, dp, 0, 2, 3, v, 1, u, &ny, y, &mv);
    ip[7] = 1;
    dp[2] = 0.01;
    s += orc_propose(h, ip, dp, 0, 3, 3, v, 0, u, &ny, y, &mv);
    // density, depths, centering rule, gradients
    double gv[9], ds[200], da[200], dg[200];
    s += orc_logp(h, 0, 3, v);
    s += orc_tau(h, 0, v, v + 3, 0) + orc_tau(h, 0, v + 3, v + 6, 1);
    s += orc_beta(h, 0, v, v + 6);
    orc_grad(h, 0, 3, v, gv, ds, da, dg);
    // anchors (low resolution) and the tracer
    for (int t = 0; t < n_targets; ++t) {
        s += orc_anchor_I2(h, t, 8, 8);
        s += orc_anchor_I3(h, t, 4, 4, 4, 4, 4);
    }
    std::vector<double> tally(2 * orc_trace_tallies());
    orc_trace(h, 0, 3, 2000, 300.0, 0.5, 2, tally.data());
    std::printf("checksum %.6g\n", s + tally[0]);
    return 0;
}

} // namespace

int main() {
    // scalar helpers
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4], r[8];
    orc_philox(ctr, key, out);
    orc_step_draws(1, 2, 3, r);
    double A[3] = {0, 0, 0}, B[3] = {1, 2, 3}, f[3], stp[3], e2[3], e3[3];
    orc_bisph(A, B, 1.0, 0.3, 2.0, f);
    orc_bisph_inv(A, B, f, stp);
    orc_onb(B, e2, e3);
    double s = orc_unif(r[0]) + orc_p_hg(0.3, 0.9) + orc_p_sl(0.3, 0.9) + orc_sigma_sr(0.3, 0.9, 0.4) +
               orc_q_s(1.0, 3.0) + orc_q_t(0.5) + orc_jac_bisph(1.0, 0.5, 2.0) + orc_kappa_eq(0.9) +
               orc_sample_cos_s(0.4, 9.0);
    std::printf("scalars %.6g\n", s);

    // homogeneous medium, vMF source, the paper's sensor response
    {
        double axis[3] = {0, 0, 1}, edges[2] = {0, 1}, ls[1] = {4.0}, la[1] = {30.0}, g[1] = {0.9}, fsl[1] = {0.0};
        int off[1] = {0}, cnt[1] = {1};
        int tmed[2] = {0, 0}, ek[2] = {1, 0}, dk[2] = {1, 0}, n0[2] = {2, 2};
        double src[6] = {0, 0, 0, 0, 0, 0}, sen[6] = {0, 0, 3.0, 0, 0.5, 3.0}, rad[2] = {0.165, 0.165};
        double ed[6] = {0, 0, 1, 0, 0, 1}, ep[2] = {4.0, 0.0}, dd[6] = {0, -1, 0, 0, -1, 0};
        void* h = orc_create(1, axis, off, cnt, edges, ls, la, g, fsl, 2, tmed, src, sen, rad, ek, ed, ep, dk, dd,
                             n0, nullptr, 16);
        exercise(h, 16, 2, 3.0);
        orc_destroy(h);
    }
    // layered medium (simplified-Liu mixture in some layers), cone source, sector tilt
    {
        const int L = 6, cap = 16;
        double axis[3] = {0, 0, 1}, edges[L + 1], ls[L], la[L], g[L], fsl[L];
        for (int l = 0; l <= L; ++l) edges[l] = -3.0 + 1.5 * l;
        for (int l = 0; l < L; ++l) {
            ls[l] = 2.0 + 0.5 * l;
            la[l] = 20.0 + 3.0 * l;
            g[l] = 0.8 + 0.02 * l;
            fsl[l] = (l % 2) ? 0.45 : 0.0;
        }
        int off[1] = {0}, cnt[1] = {L};
        int tmed[1] = {0}, ek[1] = {2}, dk[1] = {0}, n0[1] = {3};
        double src[3] = {0, 0, -1.0}, sen[3] = {0.3, 0.2, 2.0}, rad[1] = {0.165};
        double ed[3] = {0.6, 0, 0.8}, ep[1] = {0.6}, dd[3] = {0, -1, 0};
        std::vector<double> logw(cap + 1);
        for (int k = 0; k <= cap; ++k) logw[k] = 0.1 * k;
        void* h = orc_create(1, axis, off, cnt, edges, ls, la, g, fsl, 1, tmed, src, sen, rad, ek, ed, ep, dk, dd,
                             n0, logw.data(), cap);
        exercise(h, cap, 1, 3.0);
        orc_destroy(h);
    }
    return 0;
}
