// The oracle built with the sanitizers: its source compiled into a driver
// that runs one job from a file, for a run under AddressSanitizer and
// UndefinedBehaviorSanitizer (built without OpenMP, so serially).
//
//   oracle_driver <in> <out>
// in:  int32 job, int32 nsteps, float64 dt, the orc_cfg bytes, int64 nprims,
//      nprims float64 prims, int64 nextra, nextra float64 extra
//      job 0: orc_run (extra unused), 1: orc_run_face (extra = face fields),
//      2: orc_run_emhd (extra = the two extra variables), 3: orc_estimate_dt
//      and orc_divb of the prims
// out: int64 failures (job 3: 0), float64 prims, float64 extra, then
//      nsteps float64 dts (job 3: dt, divb max, divb mean)
#include "../../oracle/harm_oracle.cpp"

#include <stdio.h>
#include <stdlib.h>
#include <vector>

static void need(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "oracle_driver: %s\n", what);
    exit(2);
  }
}

int main(int argc, char** argv) {
  need(argc == 3, "usage: oracle_driver <in> <out>");
  FILE* f = fopen(argv[1], "rb");
  need(f != nullptr, "cannot open input");
  int job, nsteps;
  double dt;
  orc_cfg c;
  long np, nx;
  need(fread(&job, sizeof(int), 1, f) == 1 && fread(&nsteps, sizeof(int), 1, f) == 1 &&
           fread(&dt, sizeof(double), 1, f) == 1 && fread(&c, sizeof(c), 1, f) == 1 &&
           fread(&np, sizeof(long), 1, f) == 1,
       "short header");
  need(np > 0 && np < (1L << 28) && nsteps >= 0 && nsteps < 1000, "bad sizes");
  std::vector<double> P(np);
  need(fread(P.data(), sizeof(double), np, f) == (size_t)np && fread(&nx, sizeof(long), 1, f) == 1, "short prims");
  need(nx >= 0 && nx < (1L << 28), "bad extra size");
  std::vector<double> X(nx > 0 ? nx : 1);
  need(fread(X.data(), sizeof(double), nx, f) == (size_t)nx, "short extra");
  fclose(f);
  std::vector<double> dts(nsteps > 3 ? nsteps : 3);
  long fails = 0;
  if (job == 0)
    fails = orc_run(&c, P.data(), dt, nsteps, dts.data(), nullptr);
  else if (job == 1)
    fails = orc_run_face(&c, P.data(), X.data(), dt, nsteps, dts.data(), nullptr);
  else if (job == 2)
    fails = orc_run_emhd(&c, P.data(), X.data(), dt, nsteps, dts.data());
  else {
    need(job == 3, "bad job");
    dts[0] = orc_estimate_dt(&c, P.data());
    orc_divb(&c, P.data(), &dts[1], &dts[2], nullptr);
    nsteps = 3;
  }
  FILE* o = fopen(argv[2], "wb");
  need(o != nullptr, "cannot open output");
  need(fwrite(&fails, sizeof(long), 1, o) == 1 && fwrite(P.data(), sizeof(double), np, o) == (size_t)np &&
           fwrite(X.data(), sizeof(double), nx, o) == (size_t)nx &&
           fwrite(dts.data(), sizeof(double), nsteps, o) == (size_t)nsteps,
       "short write");
  fclose(o);
  return 0;
}
