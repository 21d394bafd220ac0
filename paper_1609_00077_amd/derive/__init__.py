"""Build-time derivation of the pair-block residual equations.

The perfect-pairing models never print their equations: the paper generates
them by machine from the spin-orbital CC equations (Sec. III, 4529 PQ and
213 234 PH contributions).  This package derives the same residuals in a
pair-site form instead.  Each pair carries four anticommuting excitation
generators (the two hole and two particle operators of its orbital quartet),
so e^{T}|0> lives in an exterior algebra, the normal-ordered Hamiltonian acts
on it by multiplication (excitation parts) and derivation (de-excitation
parts), and R = e^{-T} H_N e^{T} reduces to g_I * sum over set partitions of
derivatives of T.  Terms are enumerated with abstract pair roles (outputs P, Q;
spectators A, B, ...), which is valid for any label values because every
stored tensor is a coefficient of an operator written in role order.

Nothing here runs at solve time: the generator emits constant tables that
are compiled into the HIP library.
"""
