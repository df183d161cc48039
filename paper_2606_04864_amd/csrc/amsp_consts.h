// Compile-time constants shared by host planning and the HIP kernels.
#pragma once

namespace amsp {

constexpr int TS = 64;       // tile edge: 64x64 tiles, one wavefront-wide row block
constexpr int TE = TS * TS;  // elements per tile
// Entries of a packed diagonal factor tile: row R keeps columns 0..R, padded
// with zeros to a multiple of 4, i.e. sum over R of 4*ceil((R+1)/4).
constexpr int DE = 2176;
constexpr int WG = 256;      // workgroup size of the batched kernels (4 wavefronts)
constexpr int EIGP = 16;     // subspace block width of the local eigensolver
constexpr int MAXNEV = 15;   // nev + 1 must fit in the subspace block
constexpr int MAX_PARTIALS = 1024;  // workgroups (partial sums) of a vector reduction

}  // namespace amsp
