"""Error gates of the GPU tests (normwise relative errors, see the tests).

float64 path: 1e-12 (the bar set for the method; observed 2e-16 to 2e-15).

Mixed path (float32 hDuals, compensated sums, float64 islands): four times
the largest error measured per function on the MI355X over the mixed tests
(oracle comparisons at n = 5 .. 512, the symmetric forms, batches, float32
I/O, Ackley near x = 0):
    Rosenbrock 1.66e-7, Ackley 2.60e-7, Fletcher-Powell 2.13e-7
so the gates are 7e-7, 1.1e-6 and 9e-7.  Batches of mixed functions take
the largest.  Float32 I/O of the float64 path: its output rounding, 7.9e-8
measured, gate 3.5e-7.
"""
TOL64 = 1e-12
TOL32 = {0: 7e-7, 1: 1.1e-6, 2: 9e-7}
TOL32_ANY = max(TOL32.values())
TOL_IO32_F64 = 3.5e-7
