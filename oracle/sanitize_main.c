/*
 * sanitize_main.c -- command-line driver of the FP64 oracle for sanitizer builds.
 *
 * TEST INFRASTRUCTURE (compiled and run only by the CPU tests, with gcc's address and
 * undefined-behaviour sanitizers over vine_oracle.c).  Reads one workload written as raw
 * little-endian arrays by the test, runs vo_rollout (with the trajectory) and
 * vo_gradient on it, and writes the results as raw arrays for the test to compare with
 * the normally built oracle.
 *
 * usage: sanitize_main <in.bin> <out.bin>
 *   in.bin:  int32 B, S, O, n_steps, n_max; int32 inst_i[B][5]; double inst_d[B][6];
 *            double spam[S][4]; int32 obs_kind[O]; double obs_d[O][4]; double prm[16];
 *            double goal[B][2]
 *   out.bin: double theta[B][n_max]; double tip[B][T][3]; int32 status[B][T];
 *            uint64 chash[B][T]; double dP[S], ds0[S], ds1[S], loss[B]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int vo_rollout(int B, const int* inst_i, const double* inst_d, const double* spam,
               const int* obs_kind, const double* obs_d, const double* prm, int n_steps,
               int n_threads, int n_max, double* theta, double* tip, double* rho, int* iters,
               int* status, int* ncont, uint64_t* chash, double* maxpen, double* traj,
               double* stats, double* tiplen);
int vo_gradient(int B, const int* inst_i, const double* inst_d, const double* spam,
                const int* obs_kind, const double* obs_d, const double* prm, int T, int n_max,
                const double* traj, const double* weights, const double* goal, int n_threads,
                double* dP, double* ds0, double* ds1, double* loss);

static void* load(FILE* f, size_t size, size_t count) {
  void* p = calloc(count > 0 ? count : 1, size);
  if (!p || fread(p, size, count, f) != count) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int* hdr = (int*)load(f, sizeof(int), 5);
  const int B = hdr[0], S = hdr[1], O = hdr[2], T = hdr[3], N = hdr[4];
  int* inst_i = (int*)load(f, sizeof(int), (size_t)5 * B);
  double* inst_d = (double*)load(f, sizeof(double), (size_t)6 * B);
  double* spam = (double*)load(f, sizeof(double), (size_t)4 * S);
  int* kind = (int*)load(f, sizeof(int), (size_t)O);
  double* obs = (double*)load(f, sizeof(double), (size_t)4 * O);
  double* prm = (double*)load(f, sizeof(double), 16);
  double* goal = (double*)load(f, sizeof(double), (size_t)2 * B);
  fclose(f);
  const size_t BT = (size_t)B * T;
  double* theta = calloc((size_t)B * N, sizeof(double));
  double* tip = calloc(3 * BT, sizeof(double));
  double* rho = calloc(BT, sizeof(double));
  int* iters = calloc(BT, sizeof(int));
  int* status = calloc(BT, sizeof(int));
  int* ncont = calloc(BT, sizeof(int));
  uint64_t* chash = calloc(BT, sizeof(uint64_t));
  double* maxpen = calloc(BT, sizeof(double));
  double* traj = calloc(BT * N, sizeof(double));
  double* stats = calloc((size_t)6 * B, sizeof(double));
  vo_rollout(B, inst_i, inst_d, spam, kind, obs, prm, T, 1, N, theta, tip, rho, iters, status,
             ncont, chash, maxpen, traj, stats, NULL);
  double* dP = calloc(S + 1, sizeof(double));
  double* d0 = calloc(S + 1, sizeof(double));
  double* d1 = calloc(S + 1, sizeof(double));
  double* loss = calloc(B, sizeof(double));
  vo_gradient(B, inst_i, inst_d, spam, kind, obs, prm, T, N, traj, NULL, goal, 1, dP, d0, d1,
              loss);
  FILE* g = fopen(argv[2], "wb");
  if (!g) return 2;
  fwrite(theta, sizeof(double), (size_t)B * N, g);
  fwrite(tip, sizeof(double), 3 * BT, g);
  fwrite(status, sizeof(int), BT, g);
  fwrite(chash, sizeof(uint64_t), BT, g);
  fwrite(dP, sizeof(double), S, g);
  fwrite(d0, sizeof(double), S, g);
  fwrite(d1, sizeof(double), S, g);
  fwrite(loss, sizeof(double), B, g);
  fclose(g);
  free(hdr); free(inst_i); free(inst_d); free(spam); free(kind); free(obs); free(prm);
  free(goal); free(theta); free(tip); free(rho); free(iters); free(status); free(ncont);
  free(chash); free(maxpen); free(traj); free(stats); free(dP); free(d0); free(d1); free(loss);
  return 0;
}
