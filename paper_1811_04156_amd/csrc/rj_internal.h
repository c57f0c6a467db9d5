// rj_internal.h -- layouts shared by the host side and the kernels of
// librjpath (not part of the public ABI).
#pragma once

#include <stdint.h>

#include "../../include/rjpath.h"

namespace rj {

// Per-layer constants, LY_NW values per layer (float and double copies):
//  a, b, c = a + b, log b, g, log((1 - g^2) / (4 pi)) (HG per steradian),
//  (1 - g)^2, kappa_eq (coth k - 1/k = g), f_SL,
//  log((1 + g) / (1 - g) / (4 pi)) (SL per steradian), SL exponent 2g/(1-g).
enum {
    LY_A = 0, LY_B, LY_C, LY_LOGB, LY_G, LY_HGN, LY_HG1, LY_KEQ, LY_FSL, LY_SLN, LY_SLA,
    LY_NW = 12
};

// Per-medium description: layer offset (into the layer tables), count,
// whether the edges are uniformly spaced, the layer axis, first edge and
// inverse spacing.  Edges and prefix integrals of medium m start at
// off + m.
struct MedInfo {
    int32_t off, cnt, uniform, pad;
    double ax, ay, az, e0, inv_h;
};

// Everything a sampler launch needs, passed by value.
struct KArgs {
    // chains
    int32_t C, cap, V, prec;
    const int32_t* target;
    int32_t* n;
    void* verts;
    double* logp;
    int32_t* status;
    double* stats;
    void* work;
    // targets
    int32_t T, n_media;
    const int32_t* medium;
    const double* src;
    const double* sensor;
    const double* radius;
    const int32_t* ek;
    const double* edir;
    const double* eparam;
    const int32_t* dk;
    const double* ddir;
    const int32_t* n0;
    const double* logw;
    // media
    const MedInfo* minfo;
    const double* edge;
    const double* pre; // 2 doubles per edge: prefix of c and of b
    const void* lay;   // layer table of the chains' precision
    const double* lay64; // FP64 layer table
    int32_t L_total, n_edges;
    int32_t layered; // some medium has more than one layer
    int32_t has_sl;  // some layer has a Rayleigh-like fraction f_SL > 0
    size_t tab_bytes; // LDS bytes of the staged tables (0: read them from HBM)
    // run
    uint64_t seed, step0;
    int64_t burn_in;
    int32_t steps, cycle_len, n_perturb;
    uint32_t bthresh;
    double sigma, kappa_end, mala_h;
    int32_t sampler;
    double* trace;
    int32_t trace_steps, trace_off;
    uint32_t* hist;
    const uint64_t* step_dev; // device step counter (overrides step0) or NULL
};

} // namespace rj
