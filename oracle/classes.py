"""Oracle of the class-augmented sweep (Sec. IV-B; Prop. 2, class-augmented
value iteration) and of the class-indexed archive of Anytime-GTMP (Sec. IV-D)
for 2D point robots.

TEST INFRASTRUCTURE (see the package docstring).

Class label.  Each chosen obstacle i gets a representative point z_i (inside
the obstacle) and the upward ray {(z_x, y) : y > z_y}.  The label of a
straight edge u -> v is the vector of its signed crossings with these rays:
+1 when it crosses ray i moving in +x, -1 moving in -x, 0 otherwise.  Labels
add along concatenation, and for two start-to-goal paths that avoid the
obstacles the difference of their labels is the vector of winding numbers of
the closed loop they form around the z_i, so equal labels mean equal homology
classes (the discrete counterpart of the h-signature the paper names).

The crossing decision is defined in FP32 with a fixed operation order (no
fused multiply-add), so that a kernel taking it in FP32 takes the same one:
  straddle  (u_x < z_x) != (v_x < z_x)
  cross     = fl(fl(dx * ey) - fl(dy * ex)),  dx = v_x - u_x, dy = v_y - u_y,
              ex = z_x - u_x, ey = z_y - u_y   (each difference rounded)
  above     = cross < 0 if dx > 0 else cross > 0
  label_i   = (+1 if dx > 0 else -1) if straddle and above else 0

Sweep.  J_m(u) maps each label chi of a chain from u to the goal to the least
cost of such a chain; J over the goal layer holds the empty label with cost
0; J_m(u)[kappa(u, v) + chi] = min over v, chi of C(u, v) + J_{m+1}(v)[chi].
Edges whose cost is at least the penalty (failed edges) are absent.  The
start's map holds the least cost of every realized class.
"""
from __future__ import annotations

import itertools

import numpy as np

f32 = np.float32


def edge_label(u, v, reps):
    """Signed crossings of segment u -> v with the upward rays of reps
    [k][2] (FP32 decisions as in the module docstring): int tuple of length k."""
    ux, uy, vx, vy = f32(u[0]), f32(u[1]), f32(v[0]), f32(v[1])
    out = []
    for z in np.asarray(reps, np.float32).reshape(-1, 2):
        zx, zy = f32(z[0]), f32(z[1])
        if (ux < zx) == (vx < zx):
            out.append(0)
            continue
        dx, dy = f32(vx - ux), f32(vy - uy)
        ex, ey = f32(zx - ux), f32(zy - uy)
        cross = f32(f32(dx * ey) - f32(dy * ex))
        above = cross < 0 if dx > 0 else cross > 0
        out.append((1 if dx > 0 else -1) if above else 0)
    return tuple(out)


def add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def class_sweep(Cs, Ch, Cl, Q, q0, goals, reps, penalty):
    """Exact class-augmented backward sweep.  Returns (J_start, J) where
    J_start maps label -> (cost, chain) with chain = [i_0, ..., i_{M-1}, g]
    and J[m][u] maps label -> (cost, next vertex, next label)."""
    Q = np.asarray(Q, np.float32)
    M, N, _ = Q.shape
    goals = np.asarray(goals, np.float32).reshape(-1, 2)
    G = goals.shape[0]
    k = np.asarray(reps).reshape(-1, 2).shape[0]
    empty = (0,) * k
    J = [[dict() for _ in range(N)] for _ in range(M)]
    for u in range(N):
        for g in range(G):
            c = float(Cl[u, g])
            if not c < penalty:
                continue
            lab = add(edge_label(Q[M - 1, u], goals[g], reps), empty)
            if lab not in J[M - 1][u] or c < J[M - 1][u][lab][0]:
                J[M - 1][u][lab] = (c, g, empty)
    for m in range(M - 2, -1, -1):
        for u in range(N):
            for v in range(N):
                c = float(Ch[m, u, v])
                if not c < penalty:
                    continue
                kap = edge_label(Q[m, u], Q[m + 1, v], reps)
                for chi, (cv, _, _) in J[m + 1][v].items():
                    lab = add(kap, chi)
                    tot = c + cv
                    if lab not in J[m][u] or tot < J[m][u][lab][0]:
                        J[m][u][lab] = (tot, v, chi)
    start = {}
    for u in range(N):
        c = float(Cs[u])
        if not c < penalty:
            continue
        kap = edge_label(q0, Q[0, u], reps)
        for chi, (cv, _, _) in J[0][u].items():
            lab = add(kap, chi)
            tot = c + cv
            if lab not in start or tot < start[lab][0]:
                start[lab] = (tot, u, chi)
    out = {}
    for lab, (cost, u, chi) in start.items():
        chain = [u]
        for m in range(M):
            _, nxt, chi = J[m][chain[-1]][chi]
            chain.append(nxt)
        out[lab] = (cost, chain)
    return out, J


def chain_label_cost(Cs, Ch, Cl, Q, q0, goals, reps, chain):
    Q = np.asarray(Q, np.float32)
    goals = np.asarray(goals, np.float32).reshape(-1, 2)
    M = Q.shape[0]
    pts = [np.asarray(q0, np.float32)] + [Q[m, chain[m]] for m in range(M)] + [goals[chain[M]]]
    lab = (0,) * np.asarray(reps).reshape(-1, 2).shape[0]
    for a, b in zip(pts[:-1], pts[1:]):
        lab = add(lab, edge_label(a, b, reps))
    cost = float(Cs[chain[0]]) + sum(float(Ch[m, chain[m], chain[m + 1]]) for m in range(M - 1)) + \
        float(Cl[chain[M - 1], chain[M]])
    return lab, cost


def brute_force_classes(Cs, Ch, Cl, Q, q0, goals, reps, penalty):
    """Every chain enumerated: least cost per label (tiny graphs only)."""
    Q = np.asarray(Q, np.float32)
    M, N, _ = Q.shape
    G = np.asarray(goals).reshape(-1, 2).shape[0]
    best = {}
    for chain in itertools.product(range(N), repeat=M):
        for g in range(G):
            ch = list(chain) + [g]
            edges = [Cs[ch[0]]] + [Ch[m, ch[m], ch[m + 1]] for m in range(M - 1)] + [Cl[ch[M - 1], g]]
            if any(not float(e) < penalty for e in edges):
                continue
            lab, cost = chain_label_cost(Cs, Ch, Cl, Q, q0, goals, reps, ch)
            if lab not in best or cost < best[lab]:
                best[lab] = cost
    return best


def archive_update(archive, found, stage):
    """Class-indexed archive (Sec. IV-D): per label the lowest-cost path; a
    later stage replaces an entry only with a strictly lower cost."""
    for lab, (cost, chain) in found.items():
        if lab not in archive or cost < archive[lab][0]:
            archive[lab] = (cost, chain, stage)
    return archive


def winding_number(poly, z):
    """Winding number of a closed polygon around z by the angle sum (FP64)."""
    poly = np.asarray(poly, np.float64)
    z = np.asarray(z, np.float64)
    tot = 0.0
    for a, b in zip(poly, np.roll(poly, -1, axis=0)):
        pa, pb = a - z, b - z
        tot += np.arctan2(pa[0] * pb[1] - pa[1] * pb[0], pa @ pb)
    return int(round(tot / (2 * np.pi)))
