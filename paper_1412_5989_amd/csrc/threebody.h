// Internal interface of the three-body decoupling (threebody.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace ci {

// Device view of the coupled-JT layout and the coupling-coefficient tables.
//
// cg1: <j1 m1 j2 m2 | J M> for odd j1, j2 <= j2max (the first coupling of two
//      orbits, and of two isospins with j1 = j2 = 1).  Entry of (j1, j2):
//      cg1_off[((j1 - 1) / 2) * nj + (j2 - 1) / 2]
//        + (((m1 + j1) / 2) * (j2 + 1) + (m2 + j2) / 2) * (min(j1, j2) + 1) + (J - |j1 - j2|) / 2.
// cg2: <J12 M12 j3 m3 | J M> for even J12 <= 2 j2max and odd j3 <= j2max (the
//      second coupling).  Entry of (J12, j3):
//      cg2_off[(J12 / 2) * nj + (j3 - 1) / 2]
//        + (((M12 + J12) / 2) * (j3 + 1) + (m3 + j3) / 2) * (min(J12, j3) + 1) + (J - |J12 - j3|) / 2.
// All angular momenta doubled; FP32 values of the Racah formula.
struct ThreeBodyDev {
    int32_t nsps, nlj, ntrip, nj;  // nj = number of odd j <= j2max = 2 n1max + 1
    const uint32_t* orb;           // [nsps] orbital (n l j) | 2j << 8 | (2m + 64) << 16 | l << 24
    const int32_t* tidx;           // [nlj^3] triple index, or -1 beyond n3max
    const int64_t* block_off;      // [ntrip^2] first element of a triple pair, or -1 (parity differs)
    const int32_t* cg1_off;        // [nj][nj]
    const int32_t* cg2_off;        // [2 nj][nj]
    const float* cg1;
    const float* cg2;
};

struct ThreeBodyHost {
    int n1max = 0, n3max = 0;
    std::vector<int32_t> nlj_N, nlj_l, nlj_j2;  // oscillator orbitals (n l j)
    std::vector<int32_t> orb_alpha, orb_m2;     // m-orbits of one species
    std::vector<int32_t> tidx, trip;            // triples
    std::vector<int64_t> block_off;             // [ntrip^2]
    int64_t n_coupled = 0;
    void* arena = nullptr;
    ThreeBodyDev dev{};
};

int threebody_plan(int n1max, int n3max, ThreeBodyHost& h, std::string& err);
// <j1 m1 j2 m2 | J M> (doubled arguments) by Racah's formula in long double:
// the routine the coefficient tables are built with.
double clebsch_gordan2(int j1, int m1, int j2, int m2, int J, int M);
// Keys of the coupled elements in storage order: (t, t', 2J, 2T, 2J_ab,
// 2T_ab, 2J_de, 2T_de) per element.
void threebody_keys(const ThreeBodyHost& h, int32_t* keys);
// Device tables (one allocation, one copy).
hipError_t threebody_upload(ThreeBodyHost& h);
void threebody_release(ThreeBodyHost& h);
// work: null (requests in the given order) or decouple_work_bytes(n) bytes of
// device memory for the cost order.
size_t decouple_work_bytes(int64_t n);
hipError_t launch_decouple(const ThreeBodyHost& h, const float* A, const int32_t* req, int64_t n, void* work,
                           float* out, hipStream_t s);

}  // namespace ci
