// Internal declarations shared by the host preprocessing and the HIP entry
// points of libcgks.so.  Not part of the C ABI.
#pragma once
#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

#include "../../include/cgks.h"

namespace cgks {

// fn(begin, end) over [0, n) in contiguous chunks on up to 16 host threads.
// Used only for loops whose iterations write their own entries, so the
// results do not depend on the split.
template <class F> inline void parallel_for(int64_t n, F &&fn) {
    const unsigned hw = std::thread::hardware_concurrency();
    const int64_t nt = std::min<int64_t>(std::max(1u, std::min(hw, 16u)), std::max<int64_t>(1, n / 4096));
    if (nt <= 1) {
        fn(int64_t(0), n);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t chunk = (n + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a < b) pool.emplace_back([&fn, a, b] { fn(a, b); });
    }
    for (auto &th : pool) th.join();
}

constexpr int kMaxGP = 4;     // Gauss points per face (3-D quad)
constexpr int kMaxColoursMesh = 16;   // colour classes a caller colouring may use
constexpr int kMaxSlots = 8;  // faces per cell kept in the padded slot table
constexpr double kRankTol = 1e-8;

inline int ncoef_of(int dim) { return dim == 2 ? 5 : 9; }
inline int nquad_of(int dim) { return dim == 2 ? 3 : 6; }

// Host-side mesh: geometry in caller order plus the library cell order.
struct HostMesh {
    int dim = 0, nv = 0, nk = 0, nq = 0;
    int64_t n_cell = 0, n_face = 0, n_gp = 0, n_bface = 0;
    // input topology
    std::vector<double> xyz;
    std::vector<int64_t> fptr, fvert, owner, neigh;
    std::vector<int32_t> bc;
    std::vector<double> shift;      // [face][dim]
    // faces
    std::vector<int32_t> ngp;       // per face
    std::vector<int64_t> gp_off;    // [n_face + 1]
    std::vector<double> gx, gn, gw; // [gp][dim], [gp][dim], [gp]
    std::vector<double> avec, S;    // [face][dim], [face]
    // cells (caller order)
    std::vector<double> vol, ctr, sec, h;   // sec [cell][nq] central second moments
    std::vector<int64_t> cf_ptr, cf_face;   // faces of each cell, increasing face index
    std::vector<int8_t> cf_side;            // 0 owner, 1 neighbour
    std::vector<int32_t> colour;
    int n_colour = 0;
    // reconstruction
    std::vector<double> minv;               // [cell][nk*nk] (M^T M)^-1
    std::vector<double> gavg;               // [face][nk] ghost basis averages (boundary faces)
    // library order
    int64_t tile = 0;                       // caller cells per ordering tile
    std::vector<int64_t> lib2caller, caller2lib;
    std::vector<int64_t> colour_count;      // cells per colour
    // runs of consecutive library cells of one colour (one per tile and
    // colour present in it), grouped by colour: runs of colour c are
    // [run_ptr[c], run_ptr[c + 1])
    std::vector<int64_t> run_ptr, run_start, run_count;
    // library face order: interior faces by the smaller library index of
    // their cells, then boundary faces by their cell's (ties by caller id),
    // so a tile's faces are close together too
    std::vector<int64_t> libf2caller, caller2libf;
};

// face-based and cell-based descriptions (the latter builds the faces and
// then takes the face-based path)
cgks_status build_host_mesh(const cgks_face_mesh_desc *d, HostMesh &m);
cgks_status build_host_mesh_cells(const cgks_mesh_desc *d, HostMesh &m);

}  // namespace cgks

struct cgks_mesh {
    cgks::HostMesh hm;
};
