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
    """Rotation matrix about x (0), y (1) or z (2)."""
    c, s = np.cos(angle), np.sin(angle)
    if axis == 2:
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    if axis == 1:
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def sphere_centres(q, chain):
    """Sphere centres [S, 3] for joint angles q [7]."""
    R = np.eye(3)
    o = np.asarray(chain["base"], dtype=np.float64).copy()
    joint_R, joint_o = [], []
    for k in range(len(q)):
        R = R @ rot(int(chain["axes"][k]), q[k])
        joint_R.append(R.copy())
        joint_o.append(o.copy())
        o = o + R @ np.array([0.0, 0.0, chain["link_len"][k]])
    out = []
    for link, frac in zip(chain["sphere_link"], chain["sphere_frac"]):
        out.append(joint_o[link] + joint_R[link] @ np.array([0.0, 0.0, frac * chain["link_len"][link]]))
    return np.array(out)
