// Complex Hermitian matrices (a k-point of a periodic system) held as real
// symmetric ones.  The map phi(Z) = [[Re Z, -Im Z], [Im Z, Re Z]] keeps products,
// conjugate transposes and traces: phi(A B) = phi(A) phi(B), phi(Z^+) = phi(Z)^T,
// Tr phi(Z) = 2 Re Tr Z.  With C -> phi(C) the functional of Eq. 4 of the
// embedded problem is twice the complex one, its gradient is phi of the complex
// gradient, and CG on it from phi(C0) takes the same steps as complex CG with
// real inner products.  At block level every atom block I becomes the two
// blocks 2I (real part rows / columns) and 2I + 1 (imaginary part).  Host code.
#pragma once

#include <cstdint>
#include <vector>

#include "omm.h"

namespace omm {

// a block matrix built on the host, with an omm_matrix view of it
struct HostBlocks {
  std::vector<int32_t> rbs, cbs, ci;
  std::vector<int64_t> rp, voff;
  std::vector<double> val;
  omm_matrix m{};
  void bind();   // point m at the vectors (host memory)
};

// Block structure of a complex matrix (values not kept): nval counts complex values.
struct ZStruct {
  int nbrow = 0, nbcol = 0;
  std::vector<int32_t> rbs, cbs, ci;
  std::vector<int64_t> rp, voff;
  int64_t nval = 0;
};

// phi(Z) of a complex block matrix Z whose `val` holds 2 nval doubles (real and
// imaginary part of each value, interleaved) in host memory; Z's structure is
// recorded in zs.  Throws ArgError on a malformed Z.
void embed_complex(const omm_matrix* Z, HostBlocks& R, ZStruct& zs);

// The complex values (interleaved, 2 zs.nval doubles, in zs's layout) of the
// matrix whose embedding has the real values `real` (in the layout embed_complex
// gives for zs): Z_IJ = R(2I, 2J) + i R(2I + 1, 2J).
void extract_complex(const ZStruct& zs, const double* real, double* out);

// number of real values of the embedding of a matrix of structure zs
int64_t embedded_nval(const ZStruct& zs);

}  // namespace omm
