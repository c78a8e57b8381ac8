"""FP64 CPU oracle for the parallel Newton methods (DEER, quasi-DEER, ELK).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constants) and imports nothing from
``paper_2603_16850_amd``.

Every routine here is a plain, slow, sequential restatement of what the
thesis defines, in float64 numpy:

* ``cells``    -- the dynamics functions f(s, x) (GRU, tanh-RNN, affine), their
                  Jacobians dynamics A_t = df/ds (eq. lil_j), closed-form
                  diagonals (Ch. 3, "Efficiently Estimating the Diagonal"),
                  vector-Jacobian products and parameter gradients.
* ``rollout``  -- the sequential evaluation that defines the answer
                  (Ch. 2, Problem Statement "Unrolling an SSM", eq. ssm).
* ``newton``   -- the sequential Newton loop of Alg. alg:deer with the
                  forward-substitution update of eq. lin_rr, for any
                  transition-matrix choice of Tab. fxd_pt_sum.
* ``elk``      -- the Levenberg-Marquardt step of ELK as a sequential Kalman
                  filter (Ch. 4, Prop. prop:ELK, Sec. "Dynamics perspective on
                  ELK"), plus the associative-scan element of the parallel
                  Kalman filter the thesis cites.
* ``adjoint``  -- backpropagation through time as the reverse linear
                  recurrence of eqs. bptt / bptt_lds / unrolled_bwds.
* ``dense``    -- brute-force linear algebra on tiny problems: the block
                  bidiagonal residual Jacobian (eq. big_j), its inverse
                  (eq. J_inv), the LM step, exhaustive bracketings and the
                  up-sweep/down-sweep tree scan (Tabs. upsweep, downsweep).
* ``lle``      -- the largest-Lyapunov-exponent estimator (Alg. alg:LLE_estimate).
"""
