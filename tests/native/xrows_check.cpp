// Host check of the x-interleaved E-vector layout of the deterministic
// lattice E^T (xrows_index, xrows_width, evec_words in internal.h):
//  * every (element, local node) pair has its own word, all below evec_words;
//  * the ordered per-node sum reads, for node I = ex p + a of a lattice row,
//    word ex w + a of each candidate run and, on an x face, the word p - w
//    before it: those are exactly the words of the element nodes that
//    coincide with the lattice node.
#include <cstdio>
#include <vector>

#include "internal.h"

int main() {
  int bad = 0, cases = 0;
  for (int p = 1; p <= 8; ++p)
    for (int nx : {1, 2, 3, 5})
      for (int ny : {1, 2, 4})
        for (int nz : {1, 3}) {
          const int n = p + 1, w = pafem::xrows_width(n);
          const int64_t ne = (int64_t)nx * ny * nz, words = pafem::evec_words(ne, n);
          if (w < n || words < ne * n * n * n) ++bad;
          std::vector<int> hits(words, 0);
          for (int ez = 0; ez < nz; ++ez)
            for (int ey = 0; ey < ny; ++ey)
              for (int ex = 0; ex < nx; ++ex)
                for (int c = 0; c < n; ++c)
                  for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                      const int i = pafem::xrows_index(nx, ny, n, ex, ey, ez, a, b, c);
                      if (i < 0 || i >= words) {
                        ++bad;
                        continue;
                      }
                      ++hits[i];
                      // the sum's view of the same word: node I = ex p + a of the row
                      const int I = ex * p + a;
                      int exs = I / p, as = I - exs * p;
                      if (exs == nx) exs = nx - 1, as = p;
                      const int run = pafem::xrows_index(nx, ny, n, 0, ey, ez, 0, b, c);
                      const int col = exs * w + as;
                      const bool xface = as == 0 && exs > 0;
                      // this element's node is either the word at col or the left word
                      const bool mine = (exs == ex && as == a) ? (run + col == i)
                                        : (xface && exs == ex + 1 && a == p && run + col + p - w == i);
                      if (!mine) ++bad;
                    }
          for (int h : hits)
            if (h > 1) ++bad;
          ++cases;
        }
  std::printf("cases=%d bad=%d\n", cases, bad);
  return bad == 0 ? 0 : 1;
}
