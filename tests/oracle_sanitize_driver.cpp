// Runs every entry point of the CPU oracle once on inputs read from a file,
// for a build of the oracle with AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure only).
//
// Input file: int32 ne, n, turns, report_every; double G, gamma0, aperture;
// ne element records (the oracle's Elem layout); z[6][n], s[3][n] doubles;
// alive[n] int32.  Output file: z, s after tracking in extended precision,
// alive, the polarization reports, then the same three arrays after tracking
// in double precision, the one-turn Jacobian and quaternion derivatives of
// particle 0, and the operation counts.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
int oracle_elem_size(void);
int oracle_track(const void* el, int ne, double G, double gamma0, double aperture, int n,
                 double* z, double* s, int32_t* alive, int turns, int report_every,
                 double* pol, double* qout, int threads, int ld);
int oracle_jacobian(const void* el, int ne, double G, double gamma0, double aperture,
                    const double* z0, const double* s0, int turns, double* J, double* dQ,
                    double* zout, double* sout, double* qout);
int oracle_count_ops(const void* el, int ne, double G, double gamma0, double aperture,
                     const double* z0, int turns, long long* counts);
int oracle_romberg(const double* om, int N, double ds, int R, double* q_out, int ld);
int oracle_omega(const double* z, double h, const double* b, double G, double gamma0, double* out);
int oracle_rotate(const double* z_in, double phi, double G, double gamma0, double* z_out);
}

template <class T>
static bool get(FILE* f, T* p, size_t k) { return fread(p, sizeof(T), k, f) == k; }
template <class T>
static void put(FILE* f, const T* p, size_t k) { fwrite(p, sizeof(T), k, f); }

int main(int argc, char** argv) {
  if (argc != 3) { fprintf(stderr, "usage: %s in out\n", argv[0]); return 2; }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[4];
  double beam[3];
  if (!get(f, hdr, 4) || !get(f, beam, 3)) return 3;
  const int ne = hdr[0], n = hdr[1], turns = hdr[2], rep = hdr[3];
  const size_t esz = (size_t)oracle_elem_size();
  std::vector<unsigned char> el(esz * ne);
  std::vector<double> z(6 * (size_t)n), s(3 * (size_t)n);
  std::vector<int32_t> alive(n);
  if (!get(f, el.data(), el.size()) || !get(f, z.data(), z.size()) || !get(f, s.data(), s.size()) ||
      !get(f, alive.data(), alive.size()))
    return 3;
  fclose(f);
  const int n_rep = rep > 0 ? turns / rep : 0;
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  for (int ld = 1; ld >= 0; --ld) {
    std::vector<double> zz(z), ss(s), pol(4 * (size_t)(n_rep > 0 ? n_rep : 1)), q(4 * (size_t)n);
    std::vector<int32_t> aa(alive);
    oracle_track(el.data(), ne, beam[0], beam[1], beam[2], n, zz.data(), ss.data(), aa.data(), turns,
                 rep, pol.data(), q.data(), 2, ld);
    put(o, zz.data(), zz.size());
    put(o, ss.data(), ss.size());
    put(o, aa.data(), aa.size());
    put(o, pol.data(), 4 * (size_t)n_rep);
    put(o, q.data(), q.size());
  }
  double z0[6], s0[3] = {0.0, 1.0, 0.0}, J[36], dQ[24], zo[6], so[3], qo[4];
  for (int i = 0; i < 6; ++i) z0[i] = z[(size_t)i * n];
  oracle_jacobian(el.data(), ne, beam[0], beam[1], beam[2], z0, s0, 1, J, dQ, zo, so, qo);
  put(o, J, 36);
  put(o, dQ, 24);
  long long counts[7];
  oracle_count_ops(el.data(), ne, beam[0], beam[1], beam[2], z0, 1, counts);
  put(o, counts, 7);
  // the Romberg machinery, Ω and the face rotation on small fixed inputs
  double om[9 * 3], qr[4], oz[3], zr[6];
  for (int j = 0; j < 9; ++j) { om[3 * j] = 0.1 * j; om[3 * j + 1] = 1.0; om[3 * j + 2] = -0.2 * j; }
  oracle_romberg(om, 8, 0.5, 4, qr, 1);
  const double b[3] = {0.0, 0.05, 0.0};
  oracle_omega(z0, 0.01, b, beam[0], beam[1], oz);
  oracle_rotate(z0, 0.1, beam[0], beam[1], zr);
  put(o, qr, 4);
  put(o, oz, 3);
  put(o, zr, 6);
  fclose(o);
  return 0;
}
