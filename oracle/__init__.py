"""Plain, slow CPU oracle of the D4orm denoising hot path (FP64 NumPy).

This package is test infrastructure.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it; the product
path never does.  It shares no code with the HIP library: the only thing both
sides consume is the seeded input generator module, which holds none of the
method's arithmetic.

Modules, each following the paper's passages:
  schedule  - noise schedule alpha_i, alpha-bar_i (Section IV-B, forward process)
  noise     - the Monte Carlo sample draws (counter-based Philox4x32-10 with a
              Box-Muller transform, computed in FP32 operation by operation)
  dynamics  - RK4 rollout of the three robot models (Sections III, V)
  fitness   - team reward r(tau) and its goal / safety terms (Section IV-A),
              success and the objective (Section III)
  mbd       - batch normalisation, softmax weights, weighted mean and the
              one-step denoising update (Eqs. mc, mbd-denoising; Algorithm 1),
              the deformation iteration (Section IV-D, Algorithm 2)

Parity status of each function is stated in its docstring ("pinned by" or
"parity unpinned").
"""
