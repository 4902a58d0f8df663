// FCIDUMP reader (host code of libcdfci.so).  Molecular Hamiltonians enter
// the paper's program as FCIDUMP files with an optional truncation threshold
// on the integrals (Sec. 4.1.1 and the molecule input of Sec. 4.3); this
// turns one into the dense h and chemist (pq|rs) arrays cdfci_init takes.
//
// Format: a namelist header "&FCI NORB=n, NELEC=m, MS2=s, ORBSYM=..., ISYM=..."
// closed by "&END" or "/", then one integral per line "value i j k l" with
// 1-based orbital indices: i j k l > 0 is (ij|kl) (one of its 8 symmetric
// images), k = l = 0 is h_ij, i = j = k = l = 0 the core energy, and a line
// with only i > 0 an orbital energy (ignored).  Fortran "D" exponents are
// accepted.
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cdfci.h"

namespace {

std::string upper(std::string s) {
  for (char& ch : s) ch = (char)std::toupper((unsigned char)ch);
  return s;
}

// integer value of KEY= in the header text (first occurrence as a whole word)
bool header_int(const std::string& hdr, const char* key, long* out) {
  const std::string k = std::string(key) + "=";
  size_t pos = 0;
  while ((pos = hdr.find(k, pos)) != std::string::npos) {
    const bool word = pos == 0 || !std::isalnum((unsigned char)hdr[pos - 1]);
    if (word) {
      const char* p = hdr.c_str() + pos + k.size();
      char* end = nullptr;
      const long v = std::strtol(p, &end, 10);
      if (end == p) return false;
      *out = v;
      return true;
    }
    pos += k.size();
  }
  return false;
}

}  // namespace

extern "C" int cdfci_read_fcidump(const char* path, double threshold, int* n_orb, int* n_alpha, int* n_beta,
                                  double* h, double* eri, double* ecore) {
  if (!path || !n_orb || !n_alpha || !n_beta || threshold < 0.0) return CDFCI_ERR_INVALID_ARG;
  std::ifstream in(path);
  if (!in) return CDFCI_ERR_INVALID_ARG;
  std::string line, hdr;
  bool closed = false;
  while (std::getline(in, line)) {
    const std::string u = upper(line);
    hdr += u + " ";
    if (u.find("&END") != std::string::npos || u.find('/') != std::string::npos) {
      closed = true;
      break;
    }
  }
  if (!closed || hdr.find("&FCI") == std::string::npos) return CDFCI_ERR_INVALID_ARG;
  long norb = 0, nelec = 0, ms2 = 0;
  if (!header_int(hdr, "NORB", &norb) || !header_int(hdr, "NELEC", &nelec)) return CDFCI_ERR_INVALID_ARG;
  header_int(hdr, "MS2", &ms2);
  if (norb < 1 || nelec < 0 || ((nelec + ms2) & 1) || std::labs(ms2) > nelec) return CDFCI_ERR_INVALID_ARG;
  if (norb > 63) return CDFCI_ERR_UNSUPPORTED;
  const long na = (nelec + ms2) / 2, nb = (nelec - ms2) / 2;
  if (na > norb || nb > norb) return CDFCI_ERR_INVALID_ARG;
  *n_orb = (int)norb;
  *n_alpha = (int)na;
  *n_beta = (int)nb;
  if (!h && !eri && !ecore) return 0;
  const size_t N = (size_t)norb;
  if (h) std::memset(h, 0, N * N * sizeof(double));
  if (eri) std::memset(eri, 0, N * N * N * N * sizeof(double));
  double core = 0.0;
  while (std::getline(in, line)) {
    for (char& ch : line)
      if (ch == 'D' || ch == 'd') ch = 'E';
    std::istringstream ls(line);
    double v;
    long i, j, k, l;
    if (!(ls >> v)) continue;  // blank line
    if (!(ls >> i >> j >> k >> l)) return CDFCI_ERR_INVALID_ARG;
    if (i < 0 || j < 0 || k < 0 || l < 0 || i > norb || j > norb || k > norb || l > norb)
      return CDFCI_ERR_INVALID_ARG;
    if (!std::isfinite(v)) return CDFCI_ERR_INVALID_ARG;
    if (i == 0 && j == 0 && k == 0 && l == 0) {
      core += v;
      continue;
    }
    if (std::fabs(v) < threshold) continue;
    if (i > 0 && j > 0 && k > 0 && l > 0) {
      if (!eri) continue;
      const size_t p = i - 1, q = j - 1, r = k - 1, s = l - 1;
      const size_t img[8][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                                {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}};
      for (auto& m : img) eri[((m[0] * N + m[1]) * N + m[2]) * N + m[3]] = v;
    } else if (i > 0 && j > 0 && k == 0 && l == 0) {
      if (!h) continue;
      h[(i - 1) * N + (j - 1)] = v;
      h[(j - 1) * N + (i - 1)] = v;
    } else if (i > 0 && j == 0 && k == 0 && l == 0) {
      continue;  // orbital energy
    } else {
      return CDFCI_ERR_INVALID_ARG;
    }
  }
  if (ecore) *ecore = core;
  return 0;
}
