// Host-side exercise of the library's C ABI for the sanitizer build (AddressSanitizer
// and UndefinedBehaviorSanitizer on the host C++): meshes and their uniform refinement,
// H1 / Nedelec / L2 spaces at several orders (numbering, signs, faces, coordinates,
// boundary lists), quadrature-data sizes of every kind, and the refusal paths.  No device
// call is made.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pafem.h"

#define CHECK(x)                                                        \
  do {                                                                  \
    if (!(x)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

// n^3 lattice of the unit cube, interior vertices moved by a fixed pattern, element
// vertex order rotated per element (so every face orientation occurs)
static void lattice(int n, std::vector<double>& xyz, std::vector<int64_t>& hex) {
  const int m = n + 1;
  xyz.resize(size_t(m) * m * m * 3);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const size_t v = size_t(i + m * (j + m * k));
        const bool in = i > 0 && j > 0 && k > 0 && i < n && j < n && k < n;
        const double d = in ? 0.05 / n * std::sin(1.0 + v) : 0.0;
        xyz[3 * v + 0] = double(i) / n + d;
        xyz[3 * v + 1] = double(j) / n - d;
        xyz[3 * v + 2] = double(k) / n + 0.5 * d;
      }
  hex.clear();
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        auto V = [&](int a, int b, int c) { return int64_t(i + a + m * (j + b + m * (k + c))); };
        int64_t h[8] = {V(0, 0, 0), V(1, 0, 0), V(1, 1, 0), V(0, 1, 0),
                        V(0, 0, 1), V(1, 0, 1), V(1, 1, 1), V(0, 1, 1)};
        // rotate about z by (i + j + k) % 4 quarter turns: a relabelling that keeps det J > 0
        const int rot = (i + j + k) % 4;
        int64_t r[8];
        for (int q = 0; q < 4; ++q) {
          r[q] = h[(q + rot) % 4];
          r[4 + q] = h[4 + (q + rot) % 4];
        }
        hex.insert(hex.end(), r, r + 8);
      }
}

int main() {
  std::vector<double> xyz;
  std::vector<int64_t> hex;
  lattice(3, xyz, hex);
  const int64_t nv = int64_t(xyz.size() / 3), ne = int64_t(hex.size() / 8);
  pafem_mesh mesh = nullptr;
  CHECK(pafem_mesh_create_hex(nv, xyz.data(), ne, hex.data(), 1, nullptr, &mesh) == PAFEM_OK);
  for (int fam = 0; fam < 3; ++fam)
    for (int p = 1; p <= 8; ++p) {
      pafem_space s = nullptr;
      pafem_status st = fam == 0 ? pafem_space_create_h1(mesh, p, (p % 2) ? PAFEM_SPACE_RENUMBER : 0, &s)
                      : fam == 1 ? pafem_space_create_nd(mesh, p, 0, &s)
                                 : pafem_space_create_l2(mesh, p, 0, &s);
      CHECK(st == PAFEM_OK);
      int64_t nd = 0, nel = 0, nb = 0;
      int32_t dpe = 0, family = -1;
      CHECK(pafem_space_info(s, &nd, &nel, &dpe, &nb) == PAFEM_OK);
      CHECK(pafem_space_family(s, &family) == PAFEM_OK && family == fam);
      std::vector<int32_t> gmap(static_cast<size_t>(nel) * dpe), bdr(static_cast<size_t>(nb));
      std::vector<int8_t> sg(size_t(nel) * dpe);
      std::vector<double> X(size_t(nd) * 3);
      CHECK(pafem_space_elem_dofs(s, gmap.data()) == PAFEM_OK);
      CHECK(pafem_space_elem_signs(s, sg.data()) == PAFEM_OK);
      CHECK(pafem_space_boundary_dofs(s, bdr.data()) == PAFEM_OK);
      CHECK(pafem_space_dof_coords(s, X.data()) == PAFEM_OK);
      for (int32_t g : gmap) CHECK(g >= 0 && g < nd);
      for (int8_t v : sg) CHECK(v == 1 || v == -1);
      for (double v : X) CHECK(v > -1e-9 && v < 1.0 + 1e-9);
      size_t bytes = 0;
      CHECK(pafem_space_device_bytes(s, &bytes) == PAFEM_OK && bytes > 0);
      for (int kind = 0; kind <= 10; ++kind) {
        int64_t nq = 0;
        const pafem_status q = pafem_qdata_size(s, kind, p + 2, &nq);
        CHECK(q == PAFEM_OK || q == PAFEM_EUNSUPPORTED);
        CHECK(q != PAFEM_OK || nq > 0);
      }
      // refusals: no device image yet, bad order
      CHECK(pafem_qdata_assemble(s, PAFEM_MASS, p + 2, nullptr, 1.0, nullptr, nullptr) != PAFEM_OK);
      pafem_space_destroy(s);
    }
  // uniform refinement, twice, with the parent destroyed in between; spaces on the result
  {
    pafem_mesh f1 = nullptr, f2 = nullptr;
    CHECK(pafem_mesh_refine(mesh, &f1) == PAFEM_OK);
    CHECK(pafem_mesh_refine(f1, &f2) == PAFEM_OK);
    pafem_mesh_destroy(f1);
    int64_t fnv = 0, fne = 0;
    CHECK(pafem_mesh_info(f2, &fnv, &fne) == PAFEM_OK);
    CHECK(fne == 64 * ne && fnv == 13 * 13 * 13);
    std::vector<double> fxyz(size_t(fnv) * 3);
    std::vector<int64_t> fhex(size_t(fne) * 8);
    CHECK(pafem_mesh_vertices(f2, fxyz.data(), fhex.data()) == PAFEM_OK);
    for (int64_t v : fhex) CHECK(v >= 0 && v < fnv);
    for (double v : fxyz) CHECK(v > -1e-9 && v < 1.0 + 1e-9);
    for (int p = 1; p <= 3; ++p) {
      pafem_space s = nullptr;
      CHECK(pafem_space_create_h1(f2, p, 0, &s) == PAFEM_OK);
      int64_t nd = 0, nel = 0, nb = 0;
      int32_t dpe = 0;
      CHECK(pafem_space_info(s, &nd, &nel, &dpe, &nb) == PAFEM_OK);
      CHECK(nd == int64_t(12 * p + 1) * (12 * p + 1) * (12 * p + 1));
      pafem_space_destroy(s);
    }
    pafem_mesh_destroy(f2);
  }
  pafem_space bad = nullptr;
  CHECK(pafem_space_create_h1(mesh, 0, 0, &bad) == PAFEM_EUNSUPPORTED);
  CHECK(pafem_space_create_nd(mesh, 9, 0, &bad) == PAFEM_EUNSUPPORTED);
  CHECK(pafem_space_create_l2(mesh, -1, 0, &bad) == PAFEM_EUNSUPPORTED);
  pafem_mesh_destroy(mesh);
  // bad meshes
  std::vector<int64_t> h2 = hex;
  h2[3] = h2[2];
  pafem_mesh m2 = nullptr;
  CHECK(pafem_mesh_create_hex(nv, xyz.data(), ne, h2.data(), 1, nullptr, &m2) == PAFEM_EINVAL);
  h2 = hex;
  h2[5] = nv + 7;
  CHECK(pafem_mesh_create_hex(nv, xyz.data(), ne, h2.data(), 1, nullptr, &m2) == PAFEM_EINVAL);
  CHECK(pafem_mesh_create_hex(nv, xyz.data(), 0, hex.data(), 1, nullptr, &m2) == PAFEM_EINVAL);
  std::printf("host driver ok\n");
  return 0;
}
