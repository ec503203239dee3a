// Internal declarations of the qHP TD-CFIE library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qhp.h"

namespace qhp {

// Host description of the surface mesh and its bases (Sec. II-C, II-D).
struct Mesh {
    int64_t nv = 0, ne = 0, nc = 0;
    std::vector<double> xyz;        // [nv][3]
    std::vector<int32_t> tri;       // [nc][3]
    std::vector<int32_t> edges;     // [ne][2] (v-, v+), v- < v+
    std::vector<int32_t> cells;     // [ne][2] (c+, c-)
    std::vector<int32_t> tri_edge;  // [nc][3] edge opposite local vertex i
    std::vector<int32_t> tri_sign;  // [nc][3] +1 if the triangle is c+ of that edge
    std::vector<double> area;       // [nc]
    std::vector<int32_t> valence;   // [nv]
    double diameter = 0.0;
    int64_t n_harmonic = 0;
    // barycentric refinement
    int64_t nfv = 0, nf = 0;
    std::vector<double> fxyz;       // [nfv][3]: vertices, edge midpoints, centroids
    std::vector<int32_t> ftri;      // [nf][3]: (coarse vertex, ., .) counter-clockwise
    std::vector<int32_t> fparent;   // [nf] coarse triangle
    std::vector<int32_t> fowner;    // [nf] coarse vertex whose dual cell holds it
    // BC functions restricted to fine triangles: outward fluxes per local edge
    std::vector<int32_t> bc_off;    // [nf+1]
    std::vector<int32_t> bc_edge;   // [n_entries] BC (edge) index
    std::vector<int32_t> bc_local;  // [n_entries] rank of that edge among those of the owner vertex
    std::vector<double> bc_flux;    // [n_entries][3]
    // dual cells: fine triangles of each coarse vertex, incident edges
    std::vector<int32_t> vcell_off, vcell_tri;  // CSR over nv
    std::vector<int32_t> vedge_off, vedge;      // CSR over nv: incident edges (local rank order)
};

// Build the mesh tables; returns QHP_OK or QHP_EMESH with a message.
int build_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, Mesh &m,
               std::string &err);

// Lags: T_k = 0 for k > K (q_0 reaches two shells past the diameter).
int64_t n_lags(double diameter, double dt, int order = 1);

}  // namespace qhp
