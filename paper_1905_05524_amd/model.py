"""Algorithmic flop and byte counts of the kernels, per cell and step.

Counts follow the implemented arithmetic (FMA = 2 flops, a division = 1),
with n = N+1 nodes per direction and I Picard sweeps:

predictor, per sweep and time slice (n*n spatial nodes, 4 variables):
    gradients   2 dirs * 4 vars * n^2 outputs * n MACs      = 16 n^3
    pointwise   flux + source (FLUX_FLOPS) + gradient scaling (8)
    divergence  16 n^3, residual assembly 10 per node
    time solve  4 vars * n targets * n^2 nodes MACs         = 8 n^3
  per sweep: n * (40 n^3 + (FLUX_FLOPS + 18) n^2) + 8 n^3 (q = Q + dt acc)
  first sweep: every time slice starts from Q^n, so one slice's residual
    serves all n: 32 n^3 + (FLUX_FLOPS + 18) n^2, plus the time solve
    n * 8 n^3 + 8 n^3
  final pass: n * (16 n^3 + (FLUX_FLOPS + 8 + 28) n^2)  (28: averages)
  epilogue:   16 n^3 (volume contraction) + 64 n^2 (face values) + 16 n^2
corrector: per face node 2 eigen bounds (~14 each) + flux (4 * 4), plus the
  lifting (4 vars * 8 per node) -> small; it is bound by memory traffic.

Bytes (8-byte words, each read or written once):
  predictor: read Q (4 n^2), write Q* (4 n^2), write face data (32 n)
  corrector: read Q* (4 n^2), own and neighbour face data (64 n), write Q (4 n^2)
"""

FLUX_FLOPS = 99   # counted operation by operation in the flux/source function


def predictor_flops(N: int, iters: int = 0) -> int:
    n = N + 1
    I = iters or n
    c = FLUX_FLOPS
    slice_ = 32 * n ** 3 + (c + 18) * n ** 2     # residual of one time slice
    solve = n * 8 * n ** 3 + 8 * n ** 3           # time solve of one sweep
    sweep = n * slice_ + solve
    first = slice_ + solve                        # all slices equal Q^n
    final = n * (16 * n ** 3 + (c + 36) * n ** 2)
    epi = 16 * n ** 3 + 80 * n ** 2
    return (first + (I - 1) * sweep if I > 0 else 0) + final + epi


VJP_FLOPS = 260   # reverse of the flux/source function (forward recomputation included)


def adjoint_flops(N: int, iters: int = 0) -> int:
    """Reverse of one step per cell: the predictor recomputed with its
    iterates, then per time slice of every reverse sweep the residual
    adjoint through D^T (16 n^3), the gradients recomputed (16 n^3), the
    pointwise VJP, the gradient adjoints through D^T (16 n^3), and per sweep
    the time matrix (8 n^3 per slice); the final pass likewise without the
    residual part; the face and lifting adjoints are small."""
    n = N + 1
    I = iters or n
    c = VJP_FLOPS
    sweep = n * (48 * n ** 3 + (c + 12) * n ** 2) + 8 * n ** 4
    final = n * (32 * n ** 3 + (c + 12) * n ** 2) + 16 * n ** 3
    return predictor_flops(N, iters) + I * sweep + final + corrector_flops(N)


def corrector_flops(N: int) -> int:
    n = N + 1
    return 4 * n * (2 * 2 * 14 + 16 + 4) + 4 * n * n * 8


def step_flops(N: int, iters: int = 0) -> int:
    return predictor_flops(N, iters) + corrector_flops(N)


def predictor_bytes(N: int) -> int:
    n = N + 1
    return 8 * (8 * n * n + 32 * n)


def corrector_bytes(N: int) -> int:
    n = N + 1
    return 8 * (8 * n * n + 64 * n)


def tv_bytes(N: int) -> int:
    n = N + 1
    return 8 * (4 * n * n + 1)


def dofs(cells: int, N: int) -> int:
    return cells * (N + 1) ** 2 * 4


# ------------------------------------------------------------------------ 3D
# Three-dimensional step (n^3 nodes, 5 variables), same conventions:
# predictor, per sweep and time slice:
#     gradients   3 dirs * 5 vars * n^3 outputs * n MACs     = 30 n^4
#     pointwise   flux + source (FLUX3_FLOPS), residual scaling 6
#     divergence  30 n^4
#   per sweep: n * (60 n^4 + (FLUX3_FLOPS + 6) n^3) + 10 n^5 + 5 n^3
#     (time matrix: 5 vars * n targets * n slices MACs per node, plus Q)
#   first sweep: one slice's residual serves all n (every slice starts from
#     Q^n): 60 n^4 + (FLUX3_FLOPS + 6) n^3 + 10 n^5 + 5 n^3
#   final pass: n * (30 n^4 + (FLUX3_FLOPS + 42) n^3)   (42: 21 averages)
#   epilogue:   30 n^4 (volume term) + 15 n^3 (Q*) + 120 n^3 (60 n^2 face
#               values of n MACs)
# Bytes: predictor reads Q (5 n^3), writes Q* (5 n^3) and the face data
# (60 n^2); corrector reads Q* (5 n^3), its own and the neighbours' face
# data (120 n^2), writes Q (5 n^3) and one CFL candidate.

FLUX3_FLOPS = 180   # counted operation by operation in the 3D flux/source function


def predictor3_flops(N: int, iters: int = 0) -> int:
    n = N + 1
    I = iters or n
    c = FLUX3_FLOPS
    slice_ = 60 * n ** 4 + (c + 6) * n ** 3
    solve = 10 * n ** 5 + 5 * n ** 3
    sweep = n * slice_ + solve
    first = slice_ + solve
    final = n * (30 * n ** 4 + (c + 42) * n ** 3)
    epi = 30 * n ** 4 + 135 * n ** 3
    return (first + (I - 1) * sweep if I > 0 else 0) + final + epi


def predictor3_bytes(N: int) -> int:
    n = N + 1
    return 8 * (10 * n ** 3 + 60 * n * n)


def corrector3_bytes(N: int) -> int:
    n = N + 1
    return 8 * (10 * n ** 3 + 120 * n * n + 1)


def dofs3(cells: int, N: int) -> int:
    return cells * (N + 1) ** 3 * 5


# ------------------------------------------------------------- finite volume
# MUSCL-Hancock, per cell and step (8-byte words, each read or written once):
#   predict: read Q (4), write the evolved face values (16) and the half-step
#            density increment (1);
#   correct: read the face values of the cell and the facing values of its
#            four neighbours (32), the increment (1) and Q (4), write Q (4).
# The minimum for a step fused into one kernel is the state read and written
# once: 8 words.

def fv_predict_bytes() -> int:
    return 8 * (4 + 16 + 1)


def fv_correct_bytes() -> int:
    return 8 * (32 + 1 + 4 + 4)


def fv_min_bytes() -> int:
    return 8 * 8
