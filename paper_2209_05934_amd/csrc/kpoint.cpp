// Real embedding of complex Hermitian block matrices (k-points); see kpoint.hpp.
#include "kpoint.hpp"

#include <string>

#include "omm_internal.hpp"

namespace omm {

void HostBlocks::bind() {
  m.nbrow = (int32_t)rbs.size();
  m.nbcol = (int32_t)cbs.size();
  m.row_bsz = rbs.data();
  m.col_bsz = cbs.data();
  m.row_ptr = rp.data();
  m.col_idx = ci.data();
  m.val_off = voff.data();
  m.val = val.data();
  m.nval = (int64_t)val.size();
  m.memspace = OMM_HOST;
}

int64_t embedded_nval(const ZStruct& zs) { return 4 * zs.nval; }

void embed_complex(const omm_matrix* Z, HostBlocks& R, ZStruct& zs) {
  if (!Z) throw ArgError("complex matrix is NULL");
  if (Z->memspace != OMM_HOST) throw ArgError("complex matrices are read from host memory");
  if (Z->nbrow <= 0 || Z->nbcol <= 0 || !Z->row_bsz || !Z->col_bsz || !Z->row_ptr || !Z->col_idx ||
      !Z->val_off || !Z->val)
    throw ArgError("complex matrix: empty block structure or NULL array");
  zs.nbrow = Z->nbrow;
  zs.nbcol = Z->nbcol;
  zs.rbs.assign(Z->row_bsz, Z->row_bsz + Z->nbrow);
  zs.cbs.assign(Z->col_bsz, Z->col_bsz + Z->nbcol);
  zs.rp.assign(Z->row_ptr, Z->row_ptr + Z->nbrow + 1);
  zs.nval = Z->nval;
  for (int v : zs.rbs) if (v <= 0) throw ArgError("complex matrix: non-positive block size");
  for (int v : zs.cbs) if (v <= 0) throw ArgError("complex matrix: non-positive block size");
  if (zs.rp[0] != 0) throw ArgError("complex matrix: row_ptr[0] != 0");
  for (int i = 0; i < zs.nbrow; ++i)
    if (zs.rp[i + 1] < zs.rp[i]) throw ArgError("complex matrix: row_ptr not monotone");
  const int64_t nnzb = zs.rp[zs.nbrow];
  zs.ci.assign(Z->col_idx, Z->col_idx + nnzb);
  zs.voff.assign(Z->val_off, Z->val_off + nnzb);
  for (int i = 0; i < zs.nbrow; ++i)
    for (int64_t k = zs.rp[i]; k < zs.rp[i + 1]; ++k) {
      const int j = zs.ci[k];
      if (j < 0 || j >= zs.nbcol || (k > zs.rp[i] && zs.ci[k - 1] >= j))
        throw ArgError("complex matrix: bad column index");
      if (zs.voff[k] < 0 || zs.voff[k] + (int64_t)zs.rbs[i] * zs.cbs[j] > zs.nval)
        throw ArgError("complex matrix: val_off out of range");
    }
  // real structure: block row 2i + p holds, for each stored (i, j), blocks 2j and 2j + 1
  R.rbs.resize(2 * zs.nbrow);
  R.cbs.resize(2 * zs.nbcol);
  for (int i = 0; i < zs.nbrow; ++i) R.rbs[2 * i] = R.rbs[2 * i + 1] = zs.rbs[i];
  for (int j = 0; j < zs.nbcol; ++j) R.cbs[2 * j] = R.cbs[2 * j + 1] = zs.cbs[j];
  R.rp.assign(2 * zs.nbrow + 1, 0);
  R.ci.clear();
  R.voff.clear();
  R.val.clear();
  R.val.reserve((size_t)4 * zs.nval);
  const double* zv = Z->val;
  for (int i = 0; i < zs.nbrow; ++i)
    for (int p = 0; p < 2; ++p) {
      for (int64_t k = zs.rp[i]; k < zs.rp[i + 1]; ++k) {
        const int j = zs.ci[k], rb = zs.rbs[i], cb = zs.cbs[j];
        for (int q = 0; q < 2; ++q) {
          R.ci.push_back(2 * j + q);
          R.voff.push_back((int64_t)R.val.size());
          for (int r = 0; r < rb; ++r)
            for (int c = 0; c < cb; ++c) {
              const int64_t e = zs.voff[k] + (int64_t)r * cb + c;
              const double re = zv[2 * e], im = zv[2 * e + 1];
              // [[Re, -Im], [Im, Re]]: (p, q) = (0, 0) Re, (0, 1) -Im, (1, 0) Im, (1, 1) Re
              R.val.push_back(p == q ? re : (p == 0 ? -im : im));
            }
        }
      }
      R.rp[2 * i + p + 1] = (int64_t)R.ci.size();
    }
  R.bind();
}

void extract_complex(const ZStruct& zs, const double* real, double* out) {
  // the real values follow embed_complex's order: row 2i, then row 2i + 1, each with
  // blocks (2j, 2j + 1) per stored (i, j)
  int64_t o = 0;
  for (int i = 0; i < zs.nbrow; ++i) {
    int64_t row_len = 0;   // real values in one embedded block row 2i + p
    for (int64_t k = zs.rp[i]; k < zs.rp[i + 1]; ++k) row_len += 2 * (int64_t)zs.rbs[i] * zs.cbs[zs.ci[k]];
    const double* re_row = real + o;                // block row 2i
    const double* im_row = real + o + row_len;      // block row 2i + 1
    int64_t pos = 0;
    for (int64_t k = zs.rp[i]; k < zs.rp[i + 1]; ++k) {
      const int j = zs.ci[k], rb = zs.rbs[i], cb = zs.cbs[j];
      const int64_t sz = (int64_t)rb * cb;
      for (int64_t e = 0; e < sz; ++e) {   // block (2i, 2j) is Re Z_ij, block (2i + 1, 2j) is Im Z_ij
        out[2 * (zs.voff[k] + e)] = re_row[pos + e];
        out[2 * (zs.voff[k] + e) + 1] = im_row[pos + e];
      }
      pos += 2 * sz;   // skip block (., 2j + 1)
    }
    o += 2 * row_len;
  }
}

}  // namespace omm
