"""Pins of the blur-kernel models of the input generator: eq. (gaussian_blur) and the Gaussian-with-motion-blur
kernel of eq. (blur_kernel_final) (Sec. IV-B, App. B), against closed forms and a brute-force convolution."""
import math

import numpy as np
import pytest

from paper_2103_09943_amd import scenes


def brute_force_motion(R, sigma, d, theta, cx, cy, K=4001):
    """The continuous Gaussian averaged along the d-long segment through (cx, cy) in direction theta (midpoint
    rule with K nodes), sampled at the integer offsets and normalised to unit gain."""
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    s = (np.arange(K) + 0.5) / K * d - d / 2
    acc = np.zeros_like(xx)
    for t in s:
        px, py = cx + t * math.cos(theta), cy + t * math.sin(theta)
        acc += np.exp(-((xx - px) ** 2 + (yy - py) ** 2) / (2 * sigma ** 2))
    return acc / acc.sum()


@pytest.mark.parametrize("R,sigma,d,theta,cx,cy", [
    (9, 2.0, 3.0, math.radians(-13.7), 1.392, 0.093),  # the paper's kernel-estimation setting (Sec. IV-C)
    (4, 1.0, 1.0, 0.7, -0.3, 0.2),                       # x2 gap: 1-pixel motion, sigma 1 (Sec. IV-B)
    (8, 1.5, 5.0, 2.1, 0.0, 0.0),
])
def test_motion_blur_kernel_is_gaussian_convolved_with_segment(R, sigma, d, theta, cx, cy):
    u = scenes.motion_blur_kernel(R, sigma, d, theta, cx, cy)
    assert u.shape == (2 * R + 1, 2 * R + 1)
    assert abs(u.sum() - 1.0) < 1e-12 and u.min() >= 0.0
    np.testing.assert_allclose(u, brute_force_motion(R, sigma, d, theta, cx, cy), atol=2e-7)
    # the segment is symmetric: theta and theta + pi give one kernel
    np.testing.assert_allclose(u, scenes.motion_blur_kernel(R, sigma, d, theta + math.pi, cx, cy), atol=1e-12)


def test_motion_blur_without_motion_is_the_gaussian():
    u0 = scenes.motion_blur_kernel(6, 1.7, 0.0, 0.9, 0.4, -0.6)
    g = scenes.gaussian_kernel(13, 1.7, cx=0.4, cy=-0.6)
    np.testing.assert_allclose(u0, g, atol=1e-15)
    ue = scenes.motion_blur_kernel(6, 1.7, 1e-4, 0.9, 0.4, -0.6)  # a vanishing segment tends to it
    np.testing.assert_allclose(ue, g, atol=1e-8)


def test_gaussian_kernel_peak_and_rotation():
    """eq. (gaussian_blur): the centroid of a unit-gain sampled Gaussian with a sub-pixel peak lies at the peak
    (within the truncation), and an isotropic one does not depend on theta."""
    g = scenes.gaussian_kernel(25, 1.3, cx=0.37, cy=-0.21)
    yy, xx = np.mgrid[-12:13, -12:13]
    assert abs(float((g * xx).sum()) - 0.37) < 1e-6 and abs(float((g * yy).sum()) + 0.21) < 1e-6
    np.testing.assert_allclose(g, scenes.gaussian_kernel(25, 1.3, theta=1.1, cx=0.37, cy=-0.21), atol=1e-15)
