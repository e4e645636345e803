// TetGen mesh files (Sec. 3.2: the Node, Element and Face matrices are read
// from TetGen's .node / .ele / .face output).  Host code only.
//
//   .node  "<#points> <dim = 3> <#attributes> <#markers 0|1>", then per
//          point "<index> <x> <y> <z> [attributes...] [marker]";
//   .ele   "<#tets> <nodes per tet> <#attributes>", then
//          "<index> <n1> <n2> <n3> <n4> [further nodes] [attributes...]";
//   .face  "<#faces> <#markers 0|1>", then "<index> <n1> <n2> <n3> [marker]
//          [adjacent tets]".
// '#' starts a comment anywhere on a line.  The first point's index (0 or
// 1) is the base of every node reference.  Only linear (4-node) tets are
// accepted: the method is for T4 elements.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "common.h"

struct sfem_tetgen {
  std::string err;
  int base = 0;
  bool has_faces = false, has_markers = false;
  std::vector<double> xyz;
  std::vector<int32_t> tets, faces, markers;
};

namespace {

using sfem::Error;

// Whitespace-separated tokens of the non-comment lines of a file.
struct Lines {
  std::vector<std::vector<std::string>> rows;
};

bool read_lines(const std::string& path, Lines& out) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  while (std::getline(in, line)) {
    const size_t h = line.find('#');
    if (h != std::string::npos) line.resize(h);
    std::istringstream ss(line);
    std::vector<std::string> tok;
    std::string t;
    while (ss >> t) tok.push_back(t);
    if (!tok.empty()) out.rows.push_back(std::move(tok));
  }
  return true;
}

long long to_int(const std::string& s, const std::string& where) {
  char* end = nullptr;
  errno = 0;
  const long long v = std::strtoll(s.c_str(), &end, 10);
  if (errno || end == s.c_str() || *end) throw Error{SFEM_EINVAL, where + ": bad integer '" + s + "'"};
  return v;
}

double to_double(const std::string& s, const std::string& where) {
  char* end = nullptr;
  errno = 0;
  const double v = std::strtod(s.c_str(), &end);
  if (errno == ERANGE || end == s.c_str() || *end)
    throw Error{SFEM_EINVAL, where + ": bad number '" + s + "'"};
  return v;
}

void need(const Lines& L, size_t row, size_t ntok, const std::string& where) {
  if (row >= L.rows.size()) throw Error{SFEM_EINVAL, where + ": file ends early"};
  if (L.rows[row].size() < ntok)
    throw Error{SFEM_EINVAL, where + ": line " + std::to_string(row) + " has too few fields"};
}

void parse(sfem_tetgen& m, const std::string& stem) {
  Lines nl, el, fl;
  if (!read_lines(stem + ".node", nl)) throw Error{SFEM_EINVAL, "cannot open " + stem + ".node"};
  if (!read_lines(stem + ".ele", el)) throw Error{SFEM_EINVAL, "cannot open " + stem + ".ele"};
  m.has_faces = read_lines(stem + ".face", fl);

  const std::string wn = stem + ".node";
  need(nl, 0, 2, wn);
  const long long n = to_int(nl.rows[0][0], wn);
  const long long dim = to_int(nl.rows[0][1], wn);
  const long long nattr = nl.rows[0].size() > 2 ? to_int(nl.rows[0][2], wn) : 0;
  const long long nmark = nl.rows[0].size() > 3 ? to_int(nl.rows[0][3], wn) : 0;
  if (dim != 3) throw Error{SFEM_EINVAL, wn + ": dimension must be 3"};
  if (n <= 0 || n >= (1ll << 29) || nattr < 0 || nmark < 0 || nmark > 1)
    throw Error{SFEM_EINVAL, wn + ": bad header"};
  m.xyz.assign(size_t(3 * n), 0.0);
  std::vector<char> seen(size_t(n), 0);
  for (long long i = 0; i < n; ++i) {
    need(nl, size_t(1 + i), 4, wn);
    const auto& r = nl.rows[size_t(1 + i)];
    const long long id = to_int(r[0], wn);
    if (i == 0) {
      if (id != 0 && id != 1) throw Error{SFEM_EINVAL, wn + ": first index must be 0 or 1"};
      m.base = int(id);
    }
    const long long k = id - m.base;
    if (k < 0 || k >= n || seen[size_t(k)]) throw Error{SFEM_EINVAL, wn + ": bad point index"};
    seen[size_t(k)] = 1;
    for (int a = 0; a < 3; ++a) m.xyz[size_t(3 * k + a)] = to_double(r[size_t(1 + a)], wn);
  }

  const std::string we = stem + ".ele";
  need(el, 0, 2, we);
  const long long t = to_int(el.rows[0][0], we);
  const long long npt = to_int(el.rows[0][1], we);
  if (npt != 4) throw Error{SFEM_EINVAL, we + ": only 4-node tetrahedra are supported"};
  if (t <= 0 || t >= (1ll << 31) / 4) throw Error{SFEM_EINVAL, we + ": bad header"};
  m.tets.assign(size_t(4 * t), 0);
  for (long long i = 0; i < t; ++i) {
    need(el, size_t(1 + i), 5, we);
    const auto& r = el.rows[size_t(1 + i)];
    for (int a = 0; a < 4; ++a) {
      const long long v = to_int(r[size_t(1 + a)], we) - m.base;
      if (v < 0 || v >= n) throw Error{SFEM_EINVAL, we + ": node index out of range"};
      m.tets[size_t(4 * i + a)] = int32_t(v);
    }
  }

  if (m.has_faces) {
    const std::string wf = stem + ".face";
    need(fl, 0, 1, wf);
    const long long f = to_int(fl.rows[0][0], wf);
    const long long fm = fl.rows[0].size() > 1 ? to_int(fl.rows[0][1], wf) : 0;
    if (f < 0 || f >= (1ll << 31) / 3 || fm < 0 || fm > 1)
      throw Error{SFEM_EINVAL, wf + ": bad header"};
    m.has_markers = fm == 1;
    m.faces.assign(size_t(3 * f), 0);
    m.markers.assign(m.has_markers ? size_t(f) : 0, 0);
    for (long long i = 0; i < f; ++i) {
      need(fl, size_t(1 + i), m.has_markers ? 5 : 4, wf);
      const auto& r = fl.rows[size_t(1 + i)];
      for (int a = 0; a < 3; ++a) {
        const long long v = to_int(r[size_t(1 + a)], wf) - m.base;
        if (v < 0 || v >= n) throw Error{SFEM_EINVAL, wf + ": node index out of range"};
        m.faces[size_t(3 * i + a)] = int32_t(v);
      }
      if (m.has_markers) m.markers[size_t(i)] = int32_t(to_int(r[4], wf));
    }
  }
}

}  // namespace

extern "C" {

int sfem_tetgen_read(sfem_tetgen** out, const char* stem) {
  if (!out) return SFEM_EINVAL;
  *out = nullptr;
  sfem_tetgen* m = new (std::nothrow) sfem_tetgen();
  if (!m) return SFEM_ENOMEM;
  *out = m;
  if (!stem) {
    m->err = "null file stem";
    return SFEM_EINVAL;
  }
  try {
    parse(*m, stem);
  } catch (const Error& e) {
    m->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    m->err = e.what();
    return SFEM_ENOMEM;
  }
  return SFEM_OK;
}

const char* sfem_tetgen_last_error(const sfem_tetgen* m) { return m ? m->err.c_str() : ""; }

int sfem_tetgen_sizes(const sfem_tetgen* m, int64_t* n_nodes, int64_t* n_tets, int64_t* n_faces,
                      int* has_markers, int* index_base) {
  if (!m || !m->err.empty()) return m ? SFEM_ESTATE : SFEM_EINVAL;
  if (n_nodes) *n_nodes = int64_t(m->xyz.size() / 3);
  if (n_tets) *n_tets = int64_t(m->tets.size() / 4);
  if (n_faces) *n_faces = m->has_faces ? int64_t(m->faces.size() / 3) : -1;
  if (has_markers) *has_markers = m->has_markers ? 1 : 0;
  if (index_base) *index_base = m->base;
  return SFEM_OK;
}

int sfem_tetgen_get(const sfem_tetgen* m, double* xyz, int32_t* tets, int32_t* faces,
                    int32_t* markers) {
  if (!m || !m->err.empty()) return m ? SFEM_ESTATE : SFEM_EINVAL;
  if (xyz) std::memcpy(xyz, m->xyz.data(), m->xyz.size() * sizeof(double));
  if (tets) std::memcpy(tets, m->tets.data(), m->tets.size() * sizeof(int32_t));
  if (faces && !m->faces.empty())
    std::memcpy(faces, m->faces.data(), m->faces.size() * sizeof(int32_t));
  if (markers && !m->markers.empty())
    std::memcpy(markers, m->markers.data(), m->markers.size() * sizeof(int32_t));
  return SFEM_OK;
}

void sfem_tetgen_free(sfem_tetgen* m) { delete m; }

}  // extern "C"
