// Stand-alone driver of the host build of the kernel logic, for runs under
// AddressSanitizer and UndefinedBehaviorSanitizer with the LDS-window bounds
// check compiled in (DUGKS2P_WINDOW_CHECK).  CPU tests only.
//
// Usage: sanitize_main <case file> <output file>.  The case file holds
//   int64 kind (0: forward run, 1: rollout adjoint), steps, mseg,
//         sizeof(dugks2p_params);
//   the bytes of a dugks2p_params (its face pointers are replaced here);
//   doubles: x faces (nx + 1), y faces (ny + 1), phi0, ux0, uy0, p0
//   (nx * ny each) and, for kind 1, lam_T (18 * nx * ny).
// The output file receives, as doubles, the populations (18 * nx * ny) and
// the cell fields (5 * nx * ny) for kind 0; the final populations, the
// adjoint of phi0 (nx * ny) and the kappa / gx / gy gradient for kind 1.
#include "dugks2p_emu.cpp"

#include <stdio.h>

#include <vector>

static bool rd(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  long long hdr[4];
  dugks2p_params P;
  if (!rd(f, hdr, sizeof hdr) || hdr[3] != (long long)sizeof P || !rd(f, &P, sizeof P)) return 3;
  const size_t nx = (size_t)P.nx, ny = (size_t)P.ny, n = nx * ny;
  std::vector<double> xf(nx + 1), yf(ny + 1), in(4 * n), lam(hdr[0] == 1 ? 18 * n : 0);
  if (!rd(f, xf.data(), 8 * xf.size()) || !rd(f, yf.data(), 8 * yf.size()) ||
      !rd(f, in.data(), 8 * in.size()) || !rd(f, lam.data(), 8 * lam.size()))
    return 3;
  fclose(f);
  P.x_faces = xf.data();
  P.y_faces = yf.data();
  P.workspace = nullptr;
  const double *phi0 = in.data(), *ux0 = phi0 + n, *uy0 = ux0 + n, *p0 = uy0 + n;
  std::vector<double> out;
  int rc;
  if (hdr[0] == 0) {
    out.resize(23 * n);
    rc = emu_run(&P, phi0, ux0, uy0, p0, hdr[1], out.data(), out.data() + 18 * n);
  } else {
    out.resize(19 * n + 3);
    rc = emu_adjoint(&P, phi0, ux0, uy0, p0, hdr[1], (int)hdr[2], lam.data(), out.data(),
                     out.data() + 18 * n, out.data() + 19 * n);
  }
  if (rc) return 4;
  FILE *o = fopen(argv[2], "wb");
  if (!o || fwrite(out.data(), 8, out.size(), o) != out.size()) return 5;
  fclose(o);
  return 0;
}
