"""Plain FP64 CPU oracle for the pair-galaxy cross-correlation estimator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
It shares no code with the GPU library (no kernels, headers, tables or
helpers) and never imports it; the two meet only at the seeded catalogues
drawn by ``synth``.

What it computes (paper: Yuan, Eisenstein & Garrison 2017):
  pairs      all unordered close pairs with integer (s,|mu|) or (r_p,|pi|)
             bin keys, pair position = periodic midpoint, pair weight
             w_i w_j (Implementation section, "Mock LRG and LRG pair
             catalogue"; Methodology, the pair overdensity equation
             delta_pi_x places a pair at its midpoint);
  cic        cloud-in-cell densities on a periodic N^3 grid (the paper uses
             TSC; mass-assignment section), and TSC as a scheme;
  corr       C(r) = N_c^-1 sum_x delta_p(x) delta_g(x+r), by FFT and by a
             direct grid sum (Methodology, equation bpg_initial: the
             W-weighted average of Re(conj(dg) dp), which by Parseval is the
             real-space sum of W(r) C(r));
  bins       lattice-vector binning of C(r) into shells, (r,|mu|) or
             (r_p,|pi|), with exact lattice counts n_b;
  finalize   xi_dp from pair counts (2PCF section, equation
             2PCF_d_collapsed), b = xi_pg/xi_gg (Introduction, eq. 1),
             Q_eff (Methodology, equations Qeff and Qeff_notsq);
  grad       central finite differences and a direct-sum adjoint (no FFT)
             for gradients w.r.t. per-galaxy weights and HOD parameters;
  multipoles Legendre multipoles of xi_pg in the angle between the pair
             axis and the pair-to-galaxy direction (the other reading of the
             pair-orientation cosine), by definition and by the addition
             theorem of spherical harmonics.
"""
