// Host planner under AddressSanitizer and UndefinedBehaviorSanitizer (built with
// g++, no device code): plans for the geometries the tests use, the error
// paths, a batch cover and the real mode.  Prints one line per plan; exits
// non-zero on a failed invariant (the sanitizers abort on their own findings).
#include "plan.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>

using namespace vloc;

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAIL %s\n", what);
        ++failures;
    }
}

static void one(const int32_t grid[3], const double cell[9], double ecut, const double k[3],
                const vloc_options *opt, vloc_status want)
{
    HostPlan p;
    std::string err;
    vloc_status s = build_host_plan(p, grid, cell, ecut, k, opt, err);
    std::printf("grid %d %d %d ecut %.3f -> status %d npw %lld nst %lld groups %d %s\n", grid[0],
                grid[1], grid[2], ecut, (int)s, (long long)p.npw(), (long long)p.nst(), p.ngroups,
                err.c_str());
    expect(s == want, "status");
    if (s != VLOC_OK) return;
    long long sum = 0;
    for (const Stick &st : p.sticks) sum += st.count;
    expect(sum == p.npw(), "stick counts add up to npw");
    expect((long long)p.stick_of_slot.size() == p.nst(), "every stick has a slot");
    long long members = 0;
    for (int g = 0; g < p.ngroups; ++g) members += p.group_size[g];
    expect(members == p.nst(), "every stick is in one group");
    expect(p.holes.size() % 2 == 0, "holes are pairs");
}

int main()
{
    const double two_pi = 6.283185307179586476925286766559;
    double cubic[9] = {two_pi, 0, 0, 0, two_pi, 0, 0, 0, two_pi};
    double skew[9] = {6.0, 0.3, -0.2, 0.5, 7.0, 0.4, -0.3, 0.6, 6.5};
    double hole[9] = {4.38, 1.0686, -2.8831, 2.3836, 8.7056, -0.1596, -2.339, 2.8047, 3.0992};
    double zero_k[3] = {0, 0, 0}, kq[3] = {0.25, 1.0 / 3.0, 0}, kh[3] = {-0.3216, -0.2485, -0.2091};
    const int32_t g24[3] = {24, 24, 24}, g96[3] = {96, 96, 96}, g72[3] = {72, 96, 128};
    const int32_t g16[3] = {16, 18, 20}, gh[3] = {16, 30, 15}, g125[3] = {125, 24, 24};
    const int32_t g7[3] = {7, 24, 24}, g288[3] = {24, 24, 288};
    one(g24, cubic, 18.0, zero_k, nullptr, VLOC_OK);
    one(g96, cubic, 288.0, zero_k, nullptr, VLOC_OK);
    one(g72, cubic, 162.0, kq, nullptr, VLOC_OK);
    one(g16, skew, 12.0, kq, nullptr, VLOC_OK);
    one(gh, hole, 39.588, kh, nullptr, VLOC_OK);
    one(g125, cubic, 18.0, zero_k, nullptr, VLOC_OK);
    one(g288, cubic, 18.0, zero_k, nullptr, VLOC_OK);
    one(g7, cubic, 18.0, zero_k, nullptr, VLOC_E_GRID);
    one(g24, cubic, 72.0, zero_k, nullptr, VLOC_E_SPHERE);
    vloc_options o{};
    o.precision = VLOC_F32;
    o.deal = VLOC_DEAL_SNAKE;
    o.sticks_per_group = 5;
    one(g96, cubic, 288.0, zero_k, &o, VLOC_OK);
    vloc_options og{};
    og.gamma = 1;
    one(g96, cubic, 288.0, zero_k, &og, VLOC_OK);
    vloc_options ob{};
    ob.plane_xmode = 1;
    ob.split[0] = 12;
    one(g96, cubic, 288.0, zero_k, &ob, VLOC_OK);
    vloc_options bad{};
    bad.plane_threads = 100;
    one(g24, cubic, 18.0, zero_k, &bad, VLOC_E_INVALID);
    // a batch member widened to a larger cover
    {
        HostPlan p;
        std::string err;
        Occupied cover{-20, 20, -20, 20, -20, 20};
        vloc_status s = build_host_plan(p, g96, cubic, 162.0, kq, nullptr, err, &cover);
        expect(s == VLOC_OK && p.nxo == 41, "cover widens the occupied planes");
    }
    std::printf("%s\n", failures ? "FAILED" : "OK");
    return failures ? 1 : 0;
}
