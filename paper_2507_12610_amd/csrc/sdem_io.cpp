// File formats around the step (Section 6 of the paper, usage): meshes in
// GeomView's Object File Format with a per-face index into the list of mesh
// radii, particle states and contact springs as CSV with a header row.
// Host code only; the state is read from and written to a context through
// the ABI's own read and set calls.
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "sdem.h"

namespace {

// the library's thread-local error message lives in sdem_api.hip
int io_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

struct File {
  FILE* f = nullptr;
  explicit File(const char* path, const char* mode) : f(path ? fopen(path, mode) : nullptr) {}
  ~File() {
    if (f) fclose(f);
  }
};

// Next line without its end; false at the end of the file.
bool next_line(FILE* f, std::string& s) {
  s.clear();
  int ch;
  bool any = false;
  while ((ch = fgetc(f)) != EOF) {
    any = true;
    if (ch == '\n') break;
    if (ch != '\r') s.push_back((char)ch);
  }
  return any;
}

// Whitespace-separated tokens of a line, a '#' starting a comment.
std::vector<std::string> tokens(const std::string& line) {
  std::vector<std::string> out;
  size_t i = 0;
  const size_t n = line.find('#') == std::string::npos ? line.size() : line.find('#');
  while (i < n) {
    while (i < n && isspace((unsigned char)line[i])) ++i;
    size_t j = i;
    while (j < n && !isspace((unsigned char)line[j])) ++j;
    if (j > i) out.push_back(line.substr(i, j - i));
    i = j;
  }
  return out;
}

bool to_double(const std::string& t, double* v) {
  char* end = nullptr;
  errno = 0;
  *v = strtod(t.c_str(), &end);
  return end && *end == '\0' && end != t.c_str() && errno != ERANGE;
}

bool to_long(const std::string& t, long long* v) {
  char* end = nullptr;
  errno = 0;
  *v = strtoll(t.c_str(), &end, 10);
  return end && *end == '\0' && end != t.c_str() && errno != ERANGE;
}

std::vector<std::string> split_csv(const std::string& line) {
  std::vector<std::string> out;
  std::string cur;
  for (char ch : line) {
    if (ch == ',') {
      out.push_back(cur);
      cur.clear();
    } else if (!isspace((unsigned char)ch)) {
      cur.push_back(ch);
    }
  }
  out.push_back(cur);
  return out;
}

}  // namespace

namespace sdem {
// the ABI's error setter (defined with the context code)
int set_error(int code, const char* msg);
}  // namespace sdem

namespace {
int io_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return sdem::set_error(code, buf);
}
}  // namespace

extern "C" {

int sdem_read_off(const char* path, int32_t n_radii, const double* radii, int64_t cap,
                  int64_t* nel_out, int32_t* nverts, double* verts, double* rmesh) {
  if (!path || !nel_out) return io_fail(SDEM_EINVAL, "path and nel_out are required");
  if (n_radii < 1 || !radii) return io_fail(SDEM_EINVAL, "the list of mesh radii is empty");
  for (int32_t k = 0; k < n_radii; ++k)
    if (!(radii[k] >= 0) || !std::isfinite(radii[k]))
      return io_fail(SDEM_EINVAL, "mesh radius %d must be >= 0", k);
  File F(path, "r");
  if (!F.f) return io_fail(SDEM_EINVAL, "cannot open %s", path);
  std::string line;
  long long lineno = 0;
  // header: "OFF" (possibly followed by the counts on the same line)
  std::vector<std::string> t;
  while (t.empty() && next_line(F.f, line)) {
    ++lineno;
    t = tokens(line);
  }
  if (t.empty() || t[0] != "OFF") return io_fail(SDEM_EINVAL, "%s: no OFF header", path);
  t.erase(t.begin());
  while (t.empty() && next_line(F.f, line)) {
    ++lineno;
    t = tokens(line);
  }
  long long nv = 0, nf = 0;
  if (t.size() < 2 || !to_long(t[0], &nv) || !to_long(t[1], &nf) || nv < 0 || nf < 0)
    return io_fail(SDEM_EINVAL, "%s:%lld: expected the vertex and face counts", path, lineno);
  std::vector<double> V((size_t)nv * 3);
  for (long long i = 0; i < nv;) {
    if (!next_line(F.f, line)) return io_fail(SDEM_EINVAL, "%s: %lld vertices missing", path, nv - i);
    ++lineno;
    t = tokens(line);
    if (t.empty()) continue;
    if (t.size() < 3 || !to_double(t[0], &V[3 * i]) || !to_double(t[1], &V[3 * i + 1]) ||
        !to_double(t[2], &V[3 * i + 2]) || !std::isfinite(V[3 * i]) ||
        !std::isfinite(V[3 * i + 1]) || !std::isfinite(V[3 * i + 2]))
      return io_fail(SDEM_EINVAL, "%s:%lld: bad vertex", path, lineno);
    ++i;
  }
  int64_t nel = 0;
  for (long long f = 0; f < nf;) {
    if (!next_line(F.f, line)) return io_fail(SDEM_EINVAL, "%s: %lld faces missing", path, nf - f);
    ++lineno;
    t = tokens(line);
    if (t.empty()) continue;
    long long k = 0;
    if (!to_long(t[0], &k) || k < 1 || k > 4)
      return io_fail(SDEM_EINVAL, "%s:%lld: a face needs 1 to 4 vertices", path, lineno);
    if ((long long)t.size() < 1 + k)
      return io_fail(SDEM_EINVAL, "%s:%lld: face with missing vertex indices", path, lineno);
    long long idx[4] = {0, 0, 0, 0}, ri = 0;
    for (long long j = 0; j < k; ++j)
      if (!to_long(t[1 + j], &idx[j]) || idx[j] < 0 || idx[j] >= nv)
        return io_fail(SDEM_EINVAL, "%s:%lld: vertex index out of range", path, lineno);
    // the first number after the indices, if any, picks the mesh radius
    if ((long long)t.size() > 1 + k && (!to_long(t[1 + k], &ri) || ri < 0 || ri >= n_radii))
      return io_fail(SDEM_EINVAL, "%s:%lld: radius index not in [0, %d)", path, lineno, n_radii);
    if (nel < cap) {
      if (nverts) nverts[nel] = (int32_t)k;
      for (int j = 0; j < 4; ++j) {
        const long long v = idx[j < k ? j : k - 1];
        if (verts)
          for (int a = 0; a < 3; ++a) verts[12 * nel + 3 * j + a] = V[3 * v + a];
      }
      if (rmesh) rmesh[nel] = radii[ri];
    }
    ++nel;
    ++f;
  }
  *nel_out = nel;
  return SDEM_OK;
}

int sdem_write_csv(sdem_ctx* ctx, const char* path) {
  if (!ctx || !path) return io_fail(SDEM_EINVAL, "ctx and path are required");
  int64_t n = 0;
  int rc = sdem_spawn_status(ctx, &n, nullptr, nullptr);
  if (rc) return rc;
  std::vector<double> x(3 * n), v(3 * n), w(3 * n), q(4 * n), R(n);
  if (n) {
    if ((rc = sdem_read_state(ctx, x.data(), v.data(), w.data(), q.data(), nullptr, nullptr)))
      return rc;
    if ((rc = sdem_read_radii(ctx, R.data()))) return rc;
  }
  File F(path, "w");
  if (!F.f) return io_fail(SDEM_EINVAL, "cannot write %s", path);
  fprintf(F.f, "id,x,y,z,vx,vy,vz,wx,wy,wz,q0,q1,q2,q3,R\n");
  for (int64_t i = 0; i < n; ++i)
    fprintf(F.f,
            "%lld,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,"
            "%.17g\n",
            (long long)i, x[i], x[n + i], x[2 * n + i], v[i], v[n + i], v[2 * n + i], w[i],
            w[n + i], w[2 * n + i], q[i], q[n + i], q[2 * n + i], q[3 * n + i], R[i]);
  if (ferror(F.f)) return io_fail(SDEM_EINVAL, "write error on %s", path);
  return SDEM_OK;
}

int sdem_read_csv(const char* path, int64_t cap, int64_t* n_out, double* x, double* v, double* w,
                  double* q, double* R) {
  if (!path || !n_out) return io_fail(SDEM_EINVAL, "path and n_out are required");
  File F(path, "r");
  if (!F.f) return io_fail(SDEM_EINVAL, "cannot open %s", path);
  std::string line;
  if (!next_line(F.f, line)) return io_fail(SDEM_EINVAL, "%s: empty file", path);
  const std::vector<std::string> head = split_csv(line);
  static const char* names[15] = {"id", "x",  "y",  "z",  "vx", "vy", "vz", "wx",
                                  "wy", "wz", "q0", "q1", "q2", "q3", "R"};
  int col[15];
  for (int k = 0; k < 15; ++k) {
    col[k] = -1;
    for (size_t c = 0; c < head.size(); ++c)
      if (head[c] == names[k]) col[k] = (int)c;
  }
  for (int k : {1, 2, 3, 14})
    if (col[k] < 0) return io_fail(SDEM_EINVAL, "%s: column %s is required", path, names[k]);
  std::vector<std::vector<double>> rows;
  long long lineno = 1;
  while (next_line(F.f, line)) {
    ++lineno;
    if (tokens(line).empty()) continue;
    const std::vector<std::string> f = split_csv(line);
    std::vector<double> r(15);
    static const double dflt[15] = {-1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0};
    for (int k = 0; k < 15; ++k) {
      r[k] = dflt[k];
      if (col[k] < 0) continue;
      if ((size_t)col[k] >= f.size() || !to_double(f[col[k]], &r[k]) || !std::isfinite(r[k]))
        return io_fail(SDEM_EINVAL, "%s:%lld: bad value in column %s", path, lineno, names[k]);
    }
    if (!(r[14] > 0)) return io_fail(SDEM_EINVAL, "%s:%lld: radius must be > 0", path, lineno);
    rows.push_back(std::move(r));
  }
  const int64_t n = (int64_t)rows.size();
  // rows go to their ids when an id column is given (a permutation of 0..n-1)
  std::vector<int64_t> at((size_t)n);
  std::vector<char> seen((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t id = i;
    if (col[0] >= 0) {
      id = (int64_t)rows[i][0];
      if ((double)id != rows[i][0] || id < 0 || id >= n || seen[id])
        return io_fail(SDEM_EINVAL, "%s: the ids are not a permutation of 0..%lld", path,
                       (long long)n - 1);
      seen[id] = 1;
    }
    at[i] = id;
  }
  *n_out = n;
  if (n > cap) return SDEM_OK;  // sizes only
  for (int64_t i = 0; i < n; ++i) {
    const std::vector<double>& r = rows[i];
    const int64_t d = at[i];
    for (int k = 0; k < 3; ++k) {
      if (x) x[k * n + d] = r[1 + k];
      if (v) v[k * n + d] = r[4 + k];
      if (w) w[k * n + d] = r[7 + k];
    }
    for (int k = 0; k < 4; ++k)
      if (q) q[k * n + d] = r[10 + k];
    if (R) R[d] = r[14];
  }
  return SDEM_OK;
}

int sdem_write_contacts_csv(sdem_ctx* ctx, const char* path) {
  if (!ctx || !path) return io_fail(SDEM_EINVAL, "ctx and path are required");
  int64_t nc = 0;
  int rc = sdem_read_contacts(ctx, 0, &nc, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  std::vector<int32_t> ki(nc + 1), kj(nc + 1);
  std::vector<double> us(3 * nc + 3), ur(3 * nc + 3), ut(nc + 1);
  if (nc && (rc = sdem_read_contacts(ctx, nc, &nc, ki.data(), kj.data(), us.data(), ur.data(),
                                     ut.data())))
    return rc;
  File F(path, "w");
  if (!F.f) return io_fail(SDEM_EINVAL, "cannot write %s", path);
  fprintf(F.f, "ki,kj,usx,usy,usz,urx,ury,urz,ut\n");
  for (int64_t c = 0; c < nc; ++c)
    fprintf(F.f, "%d,%d,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g,%.17g\n", ki[c], kj[c], us[3 * c],
            us[3 * c + 1], us[3 * c + 2], ur[3 * c], ur[3 * c + 1], ur[3 * c + 2], ut[c]);
  if (ferror(F.f)) return io_fail(SDEM_EINVAL, "write error on %s", path);
  return SDEM_OK;
}

int sdem_read_contacts_csv(const char* path, int64_t cap, int64_t* nc_out, int32_t* ki,
                           int32_t* kj, double* us, double* ur, double* ut) {
  if (!path || !nc_out) return io_fail(SDEM_EINVAL, "path and nc_out are required");
  File F(path, "r");
  if (!F.f) return io_fail(SDEM_EINVAL, "cannot open %s", path);
  std::string line;
  if (!next_line(F.f, line)) return io_fail(SDEM_EINVAL, "%s: empty file", path);
  const std::vector<std::string> head = split_csv(line);
  static const char* names[9] = {"ki", "kj", "usx", "usy", "usz", "urx", "ury", "urz", "ut"};
  int col[9];
  for (int k = 0; k < 9; ++k) {
    col[k] = -1;
    for (size_t c = 0; c < head.size(); ++c)
      if (head[c] == names[k]) col[k] = (int)c;
    if (col[k] < 0) return io_fail(SDEM_EINVAL, "%s: column %s is required", path, names[k]);
  }
  int64_t nc = 0;
  long long lineno = 1;
  while (next_line(F.f, line)) {
    ++lineno;
    if (tokens(line).empty()) continue;
    const std::vector<std::string> f = split_csv(line);
    double r[9];
    for (int k = 0; k < 9; ++k)
      if ((size_t)col[k] >= f.size() || !to_double(f[col[k]], &r[k]) || !std::isfinite(r[k]))
        return io_fail(SDEM_EINVAL, "%s:%lld: bad value in column %s", path, lineno, names[k]);
    if (r[0] != std::floor(r[0]) || r[1] != std::floor(r[1]) || std::fabs(r[0]) > 2147483647.0 ||
        std::fabs(r[1]) > 2147483647.0)
      return io_fail(SDEM_EINVAL, "%s:%lld: keys must be integers", path, lineno);
    if (nc < cap) {
      if (ki) ki[nc] = (int32_t)r[0];
      if (kj) kj[nc] = (int32_t)r[1];
      for (int k = 0; k < 3; ++k) {
        if (us) us[3 * nc + k] = r[2 + k];
        if (ur) ur[3 * nc + k] = r[5 + k];
      }
      if (ut) ut[nc] = r[8];
    }
    ++nc;
  }
  *nc_out = nc;
  return SDEM_OK;
}

}  // extern "C"
