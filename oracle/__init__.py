"""Plain FP64 CPU oracle for the quasi-static projection hot path.

TEST INFRASTRUCTURE.  Nothing in the product path imports, calls or links
anything here: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library (no kernels,
headers, constants or helpers); the only thing both sides consume is the
seeded input generators in `workloads`, which hold none of the method's
arithmetic.

Written from the paper (Boffi & Rycroft, "Parallel three-dimensional
simulations of quasi-static elastoplastic solids"):

  operators.py   discrete elasticity operator (Eqs. col_snd_deriv and the
                 mixed-derivative stencil of Sec. 3.4 applied to Eq. proj),
                 staggered gradient / divergence (Eq. stag_stenc)
  multigrid.py   geometric multigrid of Sec. 3.6: trilinear T, R = T^T,
                 Galerkin A_k = R A T, V(2,2) cycle, multicolour block
                 Gauss-Seidel, dense coarsest solve
  stz.py         athermal STZ update (Eqs. stz_dpl, stz_R, stz_C_form,
                 chi_evo), intermediate stress (Eq. sig_star_qs), projection
                 step (Eqs. proj, sig_n+1)
  adjoint.py     reverse-mode derivative of a sequence of projection steps

Every array is float64; layouts follow `workloads`.
"""
