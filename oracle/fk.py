"""Forward kinematics of the synthetic 7-joint serial chain.

The paper plans for a 7-DOF WAM arm but prints no kinematic model, so the
arm is a seeded synthetic chain: joint k rotates about its local z axis
(k even) or y axis (k odd); link k extends by l_k along the rotated local z.
Frame 0 is the base translation.  Written with explicit 3x3 rotation
matrices composed joint by joint.
"""
from __future__ import annotations

import numpy as np


def rot(axis: int, angle):
    """Rotation matrix about x (0), y (1) or z (2): [3, 3] for a scalar
    angle, [..., 3, 3] for an array of angles."""
    angle = np.asarray(angle, dtype=np.float64)
    c, s = np.cos(angle), np.sin(angle)
    one, zero = np.ones_like(c), np.zeros_like(c)
    if axis == 2:
        m = [[c, -s, zero], [s, c, zero], [zero, zero, one]]
    elif axis == 1:
        m = [[c, zero, s], [zero, one, zero], [-s, zero, c]]
    else:
        m = [[one, zero, zero], [zero, c, -s], [zero, s, c]]
    return np.moveaxis(np.array(m), (0, 1), (-2, -1))


def sphere_centres(q, chain):
    """Sphere centres [S, 3] for joint angles q [7], or [K, S, 3] for a batch
    of configurations q [K, 7] (the same products, one per configuration)."""
    q = np.asarray(q, dtype=np.float64)
    Q = q.reshape(-1, q.shape[-1])
    K = Q.shape[0]
    R = np.broadcast_to(np.eye(3), (K, 3, 3)).copy()
    o = np.broadcast_to(np.asarray(chain["base"], dtype=np.float64), (K, 3)).copy()
    joint_R, joint_o = [], []
    for k in range(Q.shape[1]):
        R = R @ rot(int(chain["axes"][k]), Q[:, k])
        joint_R.append(R)
        joint_o.append(o)
        o = o + R @ np.array([0.0, 0.0, chain["link_len"][k]])
    out = np.stack([joint_o[link] + joint_R[link] @ np.array([0.0, 0.0, frac * chain["link_len"][link]])
                    for link, frac in zip(chain["sphere_link"], chain["sphere_frac"])], axis=1)
    return out[0] if q.ndim == 1 else out
