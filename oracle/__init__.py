"""CPU oracle for chunked forward-mode Hessians and Hessian-vector products.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or executes anything in this directory;
only the tests, the smoke check and the benchmark's CPU-baseline leg do.

Contents (all float64, CPU only, sharing no code with the HIP path):
  closed_form  - the plain definition: f, gradient, Hessian and H.v of the
                 three test functions written out analytically.  The chunked
                 method reaches exactly these values up to rounding, because
                 forward-mode AD on hDuals is exact differentiation (Sec. III.A,
                 Sec. III.B, Sec. IV).
  hyperdual    - brute force: the four-component hDual of Sec. III.A driven
                 by INITIALIZE and HESSIAN (n^2 calls), pure Python, tiny n.
  fd           - central finite differences, for pinning the closed forms.
  chunked      - ctypes front end of chunked.c: the paper's sequential
                 chunked method (CHUNK-INIT, CHUNK-HESS, CHESS-VEC) in plain
                 C with an instrumented operation counter (Sec. V).
"""
