// Packed form of a coarse-level plane stencil (Galerkin operator, Sec. 3.6).
//
// The full stencil of plane k holds 27 blocks of 3x3: block (oz, oy, ox)
// (each 0..2 for the offsets -1, 0, +1) couples component c of a node to
// component d of the node at that offset.  The fine operator couples c to
// d != c only through (lambda + mu) times the product of the central first
// differences along c and along d, each antisymmetric (also restricted to the
// interior planes); the transfers are tensor products, and a Galerkin product
// B^T D B of an antisymmetric factor stays antisymmetric.  So on every level
// an entry with c != d vanishes wherever the offset along c or along d is
// zero (on the grids in use such entries are rounding noise, below 1e-16 of the
// largest entry; the library checks this at setup).  Apart from the centre
// block, what remains is 150 entries per plane:
//   faces 6 x 3 (diagonal), edges 12 x 5, corners 8 x 9,
// stored in the loop order (oz, oy, ox, c, d) with unused entries skipped,
// followed by the 9 entries of the inverse centre block, the 3 diagonal
// entries of the centre block (its off-diagonal entries vanish for the same
// reason) and two pad entries.
// Kernels walk the same loops with a running index, which the compiler
// resolves to constants once the loops are unrolled.  Plain C++ (constexpr
// functions serve device code as they are), so that the host packer and its
// host check use the same definitions.
#pragma once

namespace qs {

constexpr int kPackedStencil = 164;  // entries per plane
constexpr int kPackedEntries = 150;  // off-centre entries
constexpr int kPackedInv = 150;      // 9 entries of the inverse centre block
constexpr int kPackedCentre = 159;   // 3 diagonal entries of the centre block

constexpr bool packed_used(int oz, int oy, int ox, int c, int d) {
  if (oz == 1 && oy == 1 && ox == 1) return false;
  if (c == d) return true;
  const int oc = c == 0 ? ox : (c == 1 ? oy : oz);
  const int od = d == 0 ? ox : (d == 1 ? oy : oz);
  return oc != 1 && od != 1;
}

// Position of the first packed entry of block (oz, oy, ox).
constexpr int packed_block_start(int oz, int oy, int ox) {
  int n = 0;
  for (int t = 0; t < oz * 9 + oy * 3 + ox; ++t)
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) n += packed_used(t / 9, (t / 3) % 3, t % 3, c, d) ? 1 : 0;
  return n;
}
// Packed entries of the planes oz' < oz (59 for oz = 1, 91 for oz = 2).
constexpr int packed_plane_start(int oz) { return packed_block_start(oz, 0, 0); }
static_assert(packed_plane_start(1) == 59 && packed_plane_start(2) == 91 &&
                  packed_block_start(2, 2, 2) + 9 == kPackedEntries,
              "packed stencil layout");

}  // namespace qs
