// Velocity sets and per-handle constants of the ES-BGK lattices.
//
// Storage order of the populations of every lattice: plane 0 is the rest
// velocity; velocity pair p (0 <= p < NP) occupies plane 2p+1 (velocity +c_p)
// and plane 2p+2 (velocity -c_p).  Pairs are grouped by shell, shells in
// increasing weight-table order.  The shells are those of Table I (D2Q37) and
// Table II (D2Q33) of the paper; D3Q39 uses the shells 0, (1,0,0), (1,1,1),
// (2,0,0), (2,2,0), (3,0,0).
#pragma once

#include <cstddef>
#include <cstdint>

namespace esbgk {

struct Pair {
    int c[3];
    int shell;
};

struct LatD2Q37 {
    static constexpr int D = 2, Q = 37, NP = 18, NSHELL = 8, REACH = 3;
    static constexpr Pair P[NP] = {
        {{1, 0, 0}, 1},  {{0, 1, 0}, 1},                                                   // (1,0)
        {{1, 1, 0}, 2},  {{1, -1, 0}, 2},                                                  // (1,1)
        {{2, 0, 0}, 3},  {{0, 2, 0}, 3},                                                   // (2,0)
        {{2, 1, 0}, 4},  {{1, 2, 0}, 4},  {{2, -1, 0}, 4}, {{1, -2, 0}, 4},                // (2,1)
        {{3, 0, 0}, 5},  {{0, 3, 0}, 5},                                                   // (3,0)
        {{3, 1, 0}, 6},  {{1, 3, 0}, 6},  {{3, -1, 0}, 6}, {{1, -3, 0}, 6},                // (3,1)
        {{3, 3, 0}, 7},  {{3, -3, 0}, 7},                                                  // (3,3)
    };
    // shell generators (sorted |c|) in weight-table order
    static constexpr int SHELL[NSHELL][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0},
                                             {2, 1, 0}, {3, 0, 0}, {3, 1, 0}, {3, 3, 0}};
};

struct LatD2Q33 {
    static constexpr int D = 2, Q = 33, NP = 16, NSHELL = 8, REACH = 4;
    static constexpr Pair P[NP] = {
        {{1, 0, 0}, 1}, {{0, 1, 0}, 1},                                     // (1,0)
        {{1, 1, 0}, 2}, {{1, -1, 0}, 2},                                    // (1,1)
        {{2, 0, 0}, 3}, {{0, 2, 0}, 3},                                     // (2,0)
        {{2, 2, 0}, 4}, {{2, -2, 0}, 4},                                    // (2,2)
        {{3, 0, 0}, 5}, {{0, 3, 0}, 5},                                     // (3,0)
        {{2, 1, 0}, 6}, {{1, 2, 0}, 6}, {{2, -1, 0}, 6}, {{1, -2, 0}, 6},   // (2,1)
        {{4, 4, 0}, 7}, {{4, -4, 0}, 7},                                    // (4,4)
    };
    static constexpr int SHELL[NSHELL][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0},
                                             {2, 2, 0}, {3, 0, 0}, {2, 1, 0}, {4, 4, 0}};
};

struct LatD3Q39 {
    static constexpr int D = 3, Q = 39, NP = 19, NSHELL = 6, REACH = 3;
    static constexpr Pair P[NP] = {
        {{1, 0, 0}, 1},  {{0, 1, 0}, 1},  {{0, 0, 1}, 1},                                   // (1,0,0)
        {{1, 1, 1}, 2},  {{1, 1, -1}, 2}, {{1, -1, 1}, 2}, {{-1, 1, 1}, 2},                 // (1,1,1)
        {{2, 0, 0}, 3},  {{0, 2, 0}, 3},  {{0, 0, 2}, 3},                                   // (2,0,0)
        {{2, 2, 0}, 4},  {{2, -2, 0}, 4}, {{2, 0, 2}, 4}, {{2, 0, -2}, 4},
        {{0, 2, 2}, 4},  {{0, 2, -2}, 4},                                                   // (2,2,0)
        {{3, 0, 0}, 5},  {{0, 3, 0}, 5},  {{0, 0, 3}, 5},                                   // (3,0,0)
    };
    static constexpr int SHELL[NSHELL][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 1}, {2, 0, 0}, {2, 2, 0}, {3, 0, 0}};
};

constexpr int MAX_SHELL = 8;
constexpr int MAX_Q = 39;

// Host-side constants of one lattice, in double precision.
struct LatticeConsts {
    int D = 0, Q = 0, NP = 0, nshell = 0, reach = 0;
    int c[MAX_Q][3] = {};      // storage-order velocities
    int shell_of[MAX_Q] = {};
    double wshell[MAX_SHELL] = {};
    double r = 0;
    int scale_exp[MAX_SHELL] = {};   // storage scale 2^k per shell, k = floor(log2(1/w))
};

// Fill `out` for (D, Q); returns false for an unknown lattice or a failed
// solve.  Results are computed once and cached.
bool lattice_consts(int D, int Q, LatticeConsts &out);

// Relaxation parameters (see esbgk_params in esbgk.h).  Returns 0 or
// ESBGK_EINVAL and writes a message into err.
int derive_params(int D, int Nf, double Pr, double tau, double kappa, double out[4], char *err, size_t errlen);

}  // namespace esbgk
