// Reuse of the coefficient matrix between SCF and MD steps (arXiv 2209.05934,
// Sec. III D and III E, Table 1 OMM.Extrapolate): the pattern update of a new
// geometry (blocks that left the localization radius are dropped, new ones
// start at zero), linear extrapolation from the two previous MD steps, and
// the restart file of C, whose pattern is corrected to the current one when it
// is read.  Host code only: every array here is host memory.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "omm.h"
#include "omm_internal.hpp"

namespace {

constexpr char MAGIC[8] = {'O', 'M', 'M', 'C', 'O', 'E', 'F', '1'};

// empty string when M is a well-formed host block matrix
std::string check(const omm_matrix* M, const char* name) {
  const std::string n(name);
  if (!M) return n + " is NULL";
  if (M->nbrow <= 0 || M->nbcol <= 0) return n + ": empty block structure";
  if (!M->row_bsz || !M->col_bsz || !M->row_ptr || !M->col_idx || !M->val_off || !M->val)
    return n + ": NULL array";
  if (M->memspace != OMM_HOST) return n + ": values must be in host memory";
  for (int i = 0; i < M->nbrow; ++i)
    if (M->row_bsz[i] <= 0) return n + ": non-positive row block size";
  for (int j = 0; j < M->nbcol; ++j)
    if (M->col_bsz[j] <= 0) return n + ": non-positive column block size";
  if (M->row_ptr[0] != 0) return n + ": row_ptr[0] != 0";
  for (int i = 0; i < M->nbrow; ++i) {
    if (M->row_ptr[i + 1] < M->row_ptr[i]) return n + ": row_ptr not monotone";
    for (int64_t k = M->row_ptr[i]; k < M->row_ptr[i + 1]; ++k) {
      const int j = M->col_idx[k];
      if (j < 0 || j >= M->nbcol) return n + ": column index out of range";
      if (k > M->row_ptr[i] && M->col_idx[k - 1] >= j) return n + ": columns not strictly increasing";
      const int64_t sz = (int64_t)M->row_bsz[i] * M->col_bsz[j];
      if (M->val_off[k] < 0 || M->val_off[k] + sz > M->nval) return n + ": val_off out of range";
    }
  }
  return "";
}

bool same_blocks(const omm_matrix* a, const omm_matrix* b) {
  return a->nbrow == b->nbrow && a->nbcol == b->nbcol &&
         std::memcmp(a->row_bsz, b->row_bsz, sizeof(int32_t) * a->nbrow) == 0 &&
         std::memcmp(a->col_bsz, b->col_bsz, sizeof(int32_t) * a->nbcol) == 0;
}

// stored block (i, j) of M, or -1
int64_t find_block(const omm_matrix* M, int i, int j) {
  int64_t lo = M->row_ptr[i], hi = M->row_ptr[i + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (M->col_idx[mid] < j) lo = mid + 1; else hi = mid;
  }
  return (lo < M->row_ptr[i + 1] && M->col_idx[lo] == j) ? lo : -1;
}

int fail(const std::string& msg) {
  omm::set_global_error(msg);
  return OMM_ERR_ARG;
}

int remap(const omm_matrix* cur, const omm_matrix* prev, const omm_matrix* to, double* out) {
  for (int i = 0; i < to->nbrow; ++i)
    for (int64_t k = to->row_ptr[i]; k < to->row_ptr[i + 1]; ++k) {
      const int j = to->col_idx[k];
      const int64_t sz = (int64_t)to->row_bsz[i] * to->col_bsz[j];
      double* o = out + to->val_off[k];
      const int64_t kc = find_block(cur, i, j);
      if (kc < 0) {   // a block new to the pattern starts at zero
        std::memset(o, 0, sizeof(double) * sz);
        continue;
      }
      const double* c = cur->val + cur->val_off[kc];
      const int64_t kp = prev ? find_block(prev, i, j) : -1;
      if (kp < 0) {
        std::memcpy(o, c, sizeof(double) * sz);
      } else {        // linear extrapolation 2 C_n - C_(n-1)
        const double* p = prev->val + prev->val_off[kp];
        for (int64_t e = 0; e < sz; ++e) o[e] = 2.0 * c[e] - p[e];
      }
    }
  return OMM_OK;
}

}  // namespace

extern "C" {

int omm_remap_coeffs(const omm_matrix* cur, const omm_matrix* prev, const omm_matrix* to, double* out) {
  omm::set_global_error("");
  std::string e = check(cur, "cur");
  if (e.empty() && prev) e = check(prev, "prev");
  if (e.empty()) e = check(to, "to");
  if (!e.empty()) return fail(e);
  if (!out) return fail("out is NULL");
  if (!same_blocks(cur, to) || (prev && !same_blocks(prev, to)))
    return fail("cur, prev and to must have the same block rows and columns");
  return remap(cur, prev, to, out);
}

int omm_write_coeffs(const char* path, const omm_matrix* C) {
  omm::set_global_error("");
  if (!path) return fail("path is NULL");
  const std::string e = check(C, "C");
  if (!e.empty()) return fail(e);
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(std::string("cannot open ") + path + " for writing");
  const int64_t nnzb = C->row_ptr[C->nbrow];
  int64_t nv = 0;
  std::vector<int32_t> rows(nnzb);
  for (int i = 0; i < C->nbrow; ++i)
    for (int64_t k = C->row_ptr[i]; k < C->row_ptr[i + 1]; ++k) {
      rows[k] = i;
      nv += (int64_t)C->row_bsz[i] * C->col_bsz[C->col_idx[k]];
    }
  bool ok = std::fwrite(MAGIC, 1, 8, f) == 8;
  const int32_t dims[2] = {C->nbrow, C->nbcol};
  const int64_t counts[2] = {nnzb, nv};
  ok = ok && std::fwrite(dims, sizeof(int32_t), 2, f) == 2;
  ok = ok && std::fwrite(counts, sizeof(int64_t), 2, f) == 2;
  ok = ok && std::fwrite(C->row_bsz, sizeof(int32_t), C->nbrow, f) == (size_t)C->nbrow;
  ok = ok && std::fwrite(C->col_bsz, sizeof(int32_t), C->nbcol, f) == (size_t)C->nbcol;
  ok = ok && std::fwrite(C->row_ptr, sizeof(int64_t), C->nbrow + 1, f) == (size_t)C->nbrow + 1;
  ok = ok && std::fwrite(C->col_idx, sizeof(int32_t), nnzb, f) == (size_t)nnzb;
  for (int64_t k = 0; ok && k < nnzb; ++k) {   // block values in block order, row-major
    const size_t sz = (size_t)C->row_bsz[rows[k]] * C->col_bsz[C->col_idx[k]];
    ok = std::fwrite(C->val + C->val_off[k], sizeof(double), sz, f) == sz;
  }
  ok = (std::fclose(f) == 0) && ok;
  return ok ? OMM_OK : fail(std::string("write to ") + path + " failed");
}

static int read_coeffs(const char* path, const omm_matrix* to, double* out) {
  struct File {   // closed on every way out, exceptions included
    FILE* f;
    ~File() { if (f) std::fclose(f); }
  } file{std::fopen(path, "rb")};
  FILE* f = file.f;
  if (!f) return fail(std::string("cannot open ") + path);
  auto bad = [&](const char* what) { return fail(std::string(path) + ": " + what); };
  char magic[8];
  int32_t dims[2];
  int64_t counts[2];
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, MAGIC, 8) != 0) return bad("not a coefficient file");
  if (std::fread(dims, sizeof(int32_t), 2, f) != 2 || std::fread(counts, sizeof(int64_t), 2, f) != 2)
    return bad("truncated header");
  if (dims[0] != to->nbrow || dims[1] != to->nbcol) return bad("block rows/columns differ from the target's");
  const int64_t nnzb = counts[0], nv = counts[1];
  if (nnzb < 0 || nnzb > (int64_t)dims[0] * dims[1] || nv < 0) return bad("corrupt counts");
  // block sizes first: they must be the target's, which bounds every size read after them
  std::vector<int32_t> rbs(dims[0]), cbs(dims[1]);
  if (std::fread(rbs.data(), sizeof(int32_t), dims[0], f) != (size_t)dims[0] ||
      std::fread(cbs.data(), sizeof(int32_t), dims[1], f) != (size_t)dims[1])
    return bad("truncated structure");
  for (int i = 0; i < dims[0]; ++i)
    if (rbs[i] != to->row_bsz[i]) return bad("block sizes differ from the target's");
  for (int j = 0; j < dims[1]; ++j)
    if (cbs[j] != to->col_bsz[j]) return bad("block sizes differ from the target's");
  std::vector<int32_t> ci(nnzb);
  std::vector<int64_t> rp(dims[0] + 1), voff(nnzb);
  if (std::fread(rp.data(), sizeof(int64_t), dims[0] + 1, f) != (size_t)dims[0] + 1 ||
      std::fread(ci.data(), sizeof(int32_t), nnzb, f) != (size_t)nnzb)
    return bad("truncated structure");
  if (rp[0] != 0 || rp[dims[0]] != nnzb) return bad("corrupt row pointers");
  int64_t o = 0;
  for (int i = 0; i < dims[0]; ++i) {
    if (rp[i + 1] < rp[i]) return bad("corrupt row pointers");
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= dims[1]) return bad("corrupt column index");
      voff[k] = o;
      o += (int64_t)rbs[i] * cbs[ci[k]];
    }
  }
  // the value count follows from the structure; only a file that agrees with it is read on
  if (o != nv) return bad("value count does not match the blocks");
  std::vector<double> val(nv);
  if (std::fread(val.data(), sizeof(double), nv, f) != (size_t)nv) return bad("truncated values");
  omm_matrix src{};
  src.nbrow = dims[0];
  src.nbcol = dims[1];
  src.row_bsz = rbs.data();
  src.col_bsz = cbs.data();
  src.row_ptr = rp.data();
  src.col_idx = ci.data();
  src.val_off = voff.data();
  src.val = val.data();
  src.nval = nv;
  src.memspace = OMM_HOST;
  const std::string es = check(&src, path);
  if (!es.empty()) return fail(es);
  if (!same_blocks(&src, to)) return fail(std::string(path) + ": block sizes differ from the target's");
  return remap(&src, nullptr, to, out);
}

int omm_read_coeffs(const char* path, const omm_matrix* to, double* out) {
  omm::set_global_error("");
  if (!path) return fail("path is NULL");
  const std::string e = check(to, "to");
  if (!e.empty()) return fail(e);
  if (!out) return fail("out is NULL");
  try {   // no C++ exception leaves the C ABI
    return read_coeffs(path, to, out);
  } catch (const std::bad_alloc&) {
    omm::set_global_error(std::string(path) + ": host allocation failed");
    return OMM_ERR_OOM;
  } catch (...) {
    return fail(std::string(path) + ": unreadable coefficient file");
  }
}

}  // extern "C"
